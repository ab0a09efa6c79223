// FP32 instantiations of the line-kernel classes with a kernel extension
// (iterated closures, Runge-Kutta stage epilogue, accumulating store; see
// cfd_lines.h), compiled on their own so the build runs them in parallel.
#include <hip/hip_runtime.h>

#include "cfd_internal.h"
#include "cfd_lines.h"
#include "cfd_kernels_reg.h"

namespace cfd {
extern const LineClass kLineClassesExtF32[] = {CFD_LINE_CLASSES_EXT(float, 1)};
extern const int kNumLineClassesExtF32 = (int)(sizeof(kLineClassesExtF32) / sizeof(kLineClassesExtF32[0]));
}  // namespace cfd
