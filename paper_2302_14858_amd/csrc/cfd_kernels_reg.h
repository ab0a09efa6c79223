// Registry of compiled line-kernel classes (shared by the FP64 and FP32
// instantiation units).  A class fixes the band (nl), the operators fused in
// one pass (nops), their parities (par), the interior stencil half-width (mi)
// and the ring half-width (hw); each compiled kernel carries a set of
// partition lengths L chosen per work item.
#pragma once

#include "cfd_internal.h"

namespace cfd {

struct LineClass {
    int nl, nops, par, mi, hw;
    int nL;
    int Ls[8];
    const void *fn;
    int ext;      // extension mode: 1 end-value terms of an iterated closure, 2 stage epilogue, 3 accumulate
    int wg;       // wavefronts per workgroup: 4 (P = 1, 2, 4) or 8 (P = 8)
};

#define CFD_LC(T, NL, NOPS, PAR, MI, HW, ...)                                                        \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 0, 4, __VA_ARGS__>), 0, 4}
#define CFD_LC8(T, NL, NOPS, PAR, MI, HW, ...)                                                       \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 0, 8, __VA_ARGS__>), 0, 8}
#define CFD_LC_EXT(T, NL, NOPS, PAR, MI, HW, ...)                                                    \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 1, 4, __VA_ARGS__>), 1, 4}
#define CFD_LC_RK(T, NL, NOPS, PAR, MI, HW, ...)                                                     \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 2, 4, __VA_ARGS__>), 2, 4}
#define CFD_LC_ACC(T, NL, NOPS, PAR, MI, HW, ...)                                                    \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 3, 4, __VA_ARGS__>), 3, 4}
#define CFD_LC8_ACC(T, NL, NOPS, PAR, MI, HW, ...)                                                   \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 3, 8, __VA_ARGS__>), 3, 8}
#define CFD_LC8_RK(T, NL, NOPS, PAR, MI, HW, ...)                                                    \
    LineClass{NL, NOPS, PAR, MI, HW, LSet<__VA_ARGS__>::n, {__VA_ARGS__},                              \
              reinterpret_cast<const void *>(&k_lines<T, NL, NOPS, PAR, MI, HW, 2, 8, __VA_ARGS__>), 2, 8}

// The classes compiled for each precision.
#define CFD_LINE_CLASSES(T, F32)                                                  \
    /* pentadiagonal, first + second derivative, RHS half-width 3, closures 5; */ \
    /* the class without 24-row partitions needs fewer registers (4 waves per */  \
    /* SIMD instead of 3) and is preferred for the lengths it has */              \
    CFD_LC(T, 2, 2, 1, 3, 5, 8, 12, 16),                                          \
    CFD_LC(T, 2, 2, 1, 3, 5, 8, 12, 16, 24),                                      \
    /* tridiagonal, first + second derivative, RHS half-width 3, closures 4 */    \
    CFD_LC(T, 1, 2, 1, 3, 4, 8, 12, 16),                                          \
    CFD_LC(T, 1, 2, 1, 3, 4, 8, 12, 16, 24, 32),                                  \
    /* tridiagonal first derivative, RHS half-width 3 (short and long lines) */   \
    CFD_LC(T, 1, 1, 1, 3, 4, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 1, 1, 1, 3, 4, 48, 64),                                             \
    /* tridiagonal second derivative alone, RHS half-width up to 3 (short and   */ \
    /* long lines)                                                              */ \
    CFD_LC(T, 1, 1, 0, 3, 4, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 1, 1, 0, 3, 4, 48, 64),                                             \
    /* tridiagonal first derivative, RHS half-width 2 */                          \
    CFD_LC(T, 1, 1, 1, 2, 4, 8, 16, 32, 64),                                      \
    /* any single operator with stencils up to half-width 5 */                    \
    CFD_LC(T, 1, 1, 1, 5, 5, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 1, 1, 0, 5, 5, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 2, 1, 1, 5, 5, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 2, 1, 0, 5, 5, 8, 12, 16, 24, 32),                                  \
    /* explicit schemes */                                                        \
    CFD_LC(T, 0, 1, 1, 5, 5, 8, 12, 16, 24, 32),                                  \
    CFD_LC(T, 0, 1, 0, 5, 5, 8, 12, 16, 24, 32),                                  \
    /* long lines in 8 partitions (8-wave workgroups): tridiagonal first +     */ \
    /* second derivative (16-row partitions alone keep 4 waves per SIMD), and  */ \
    /* first or second derivative alone, partitions of 16..32 rows             */ \
    CFD_LC8(T, 1, 2, 1, 3, 4, 16),                                                \
    CFD_LC8(T, 1, 2, 1, 3, 4, 16, 24, 32),                                        \
    CFD_LC8(T, 1, 1, 1, 3, 4, 16, 24, 32),                                        \
    CFD_LC8(T, 1, 1, 0, 3, 4, 16, 24, 32)

// The classes with a kernel extension, compiled in translation units of their
// own (cfd_kernels_ext*.hip) so that the build runs more of them in parallel.
#define CFD_LINE_CLASSES_EXT(T, F32)                                              \
    /* iterated closures of tridiagonal schemes (hybrid closure iteration) */    \
    CFD_LC_EXT(T, 1, 2, 1, 3, 4, 8, 12, 16),                                      \
    CFD_LC_EXT(T, 1, 1, 1, 3, 4, 8, 12, 16, 24, 32),                              \
    CFD_LC_EXT(T, 1, 1, 0, 5, 5, 8, 12, 16, 24, 32),                              \
    /* the fused Runge-Kutta stage of the wave system (tridiagonal first      */ \
    /* derivatives with RHS half-width up to 3), the partition sets of the     */ \
    /* plain classes above; the class without long partitions needs fewer      */ \
    /* registers and is preferred for the lengths it has                       */ \
    CFD_LC_RK(T, 1, 1, 1, 3, 4, 8, 12, 16),                                       \
    CFD_LC_RK(T, 1, 1, 1, 3, 4, 8, 12, 16, 24, 32),                               \
    CFD_LC8_RK(T, 1, 1, 1, 3, 4, 16, 24, 32),                                     \
    /* accumulating first derivatives: the second order of the symmetrised     */ \
    /* mixed derivatives (explicit, tri- and pentadiagonal; long tri lines)     */ \
    CFD_LC_ACC(T, 0, 1, 1, 5, 5, 8, 12, 16, 24, 32),                              \
    CFD_LC_ACC(T, 1, 1, 1, 5, 5, 8, 12, 16, 24, 32),                              \
    CFD_LC_ACC(T, 2, 1, 1, 5, 5, 8, 12, 16, 24, 32),                              \
    CFD_LC8_ACC(T, 1, 1, 1, 3, 4, 16, 24, 32)

const LineClass *find_line_class(int f32, int nl, int nops, int par, int mi, int hw, int L, int ext, int wg);

// The tables, one per precision and translation unit.
extern const LineClass kLineClassesF64[];
extern const int kNumLineClassesF64;
extern const LineClass kLineClassesF32[];
extern const int kNumLineClassesF32;
extern const LineClass kLineClassesExtF64[];
extern const int kNumLineClassesExtF64;
extern const LineClass kLineClassesExtF32[];
extern const int kNumLineClassesExtF32;

}  // namespace cfd
