// FP32 instantiations of the line kernel (cfd_lines.h), compiled on their own
// so the two precisions build in parallel.
#include <hip/hip_runtime.h>

#include "cfd_internal.h"
#include "cfd_lines.h"
#include "cfd_kernels_reg.h"

namespace cfd {
extern const LineClass kLineClassesF32[] = {CFD_LINE_CLASSES(float, 1)};
extern const int kNumLineClassesF32 = (int)(sizeof(kLineClassesF32) / sizeof(kLineClassesF32[0]));
}  // namespace cfd
