// Hybrid iteration of the block closures (arXiv 2302.14858,
// Sec. ssec:domdec_iter, Eq. iter_center_P and its matrix form Eq. iter_scheme).
//
// On a periodic lattice of blocks, iterate i > 0 of a tridiagonal scheme solves
// each block line with the derivative two nodes past either end fixed to the
// neighbouring block's iterate i - 1 there.  Written on the block's own nodes
// (the host's make_iterated), that is a closure system with implicit closure
// rows whose right side carries gamma times each end value, so
//   x^[i] = xf + e-^[i-1] g- + e+^[i-1] g+,
// with xf the solution for zero end values and g-, g+ fixed influence vectors.
// Only two values per line pass between the blocks: the iterate at nodes c - 1
// and N - c (c = 2), which the neighbours read as their end values.  The
// device work per apply:
//   1. k_end_values: per line, the iterate-0 values at those nodes (the block
//      closure of Eq. sch_cent_om) and the xf values there, as dot products of
//      the line with rows of h^-d D_L^-1 D_R built once per plan
//      (k_end_weights, FP64);
//   2. k_iter_ends, step: the end-node values of the next iterate from the
//      neighbours' current ones (no pass over the fields); gather: each line's
//      two end values for the last iterate;
//   3. the line kernel of the iterated system (EXT class), which adds
//      e- g- + e+ g+ to its solution.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

// One weight table: both systems of one (scheme, N), FP64.
struct EndWeightSpec {
    int N, c, d;                 // line length, end-node offset, derivative degree
    double alpha;                // interior alpha^(d)_{+-1}
    double a[2 * kMaxHalf + 1];  // interior stencil
    double cl[2 * kMaxHalf + 1]; // block-closure stencil of row k*_- (identity row of D_L)
    double ce[2 * kMaxHalf + 1]; // iterated closure stencil of row k*_-
    double cl_d0, cl_up;         // iterated closure row of D_L
    int64_t off;                 // output: 4 x (N + 2 kMaxHalf) doubles
};

// Row `row` of D_R (stencil centred at node row, over nodes -R .. N+R-1) of
// system ext (0: block closure, 1: iterated closure), accumulated with weight z.
__device__ inline void add_dr_row(const EndWeightSpec &s, int ext, int row, double z, double *w) {
    constexpr int R = kMaxHalf;
    const double sgn = (s.d % 2) ? -1.0 : 1.0;
    const double *st;
    bool mirror = false;
    if (row == 0) st = ext ? s.ce : s.cl;
    else if (row == s.N - 1) { st = ext ? s.ce : s.cl; mirror = true; }
    else st = s.a;
    for (int m = -R; m <= R; ++m) {
        const double v = mirror ? sgn * st[R - m] : st[R + m];
        if (v != 0.0) w[row + m + R] += z * v;
    }
}

// Thread (table, q): q = 0, 1 block closure at rows c - 1, N - c; q = 2, 3 the
// iterated system at the same rows.  Row j of D_L^-1 D_R is z^T D_R with
// D_L^T z = e_j, a tridiagonal solve without pivoting.
__global__ void k_end_weights(int ntab, const EndWeightSpec *__restrict__ specs, double *__restrict__ data,
                              double *__restrict__ scratch, int stride) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * ntab) return;
    const EndWeightSpec s = specs[t / 4];
    const int q = t % 4;
    const int ext = q >= 2;
    const int N = s.N;
    const int j = (q % 2) ? N - s.c : s.c - 1;
    double *cp = scratch + (int64_t)t * 2 * stride;   // stride >= every table's N
    double *z = cp + N;
    // D_L rows: (lo, di, up)
    auto lo = [&](int r) -> double {
        if (r == 0) return 0.0;
        if (r == N - 1) return ext ? s.cl_up : 0.0;
        return s.alpha;
    };
    auto up = [&](int r) -> double {
        if (r == N - 1) return 0.0;
        if (r == 0) return ext ? s.cl_up : 0.0;
        return s.alpha;
    };
    auto di = [&](int r) -> double { return (r == 0 || r == N - 1) ? (ext ? s.cl_d0 : 1.0) : 1.0; };
    // D_L^T: sub-diagonal up(r-1), diagonal di(r), super-diagonal lo(r+1)
    for (int r = 0; r < N; ++r) {
        const double sub = r > 0 ? up(r - 1) : 0.0;
        const double sup = r + 1 < N ? lo(r + 1) : 0.0;
        const double rhs = r == j ? 1.0 : 0.0;
        const double m = di(r) - (r > 0 ? sub * cp[r - 1] : 0.0);
        cp[r] = sup / m;
        z[r] = (rhs - (r > 0 ? sub * z[r - 1] : 0.0)) / m;
    }
    for (int r = N - 2; r >= 0; --r) z[r] -= cp[r] * z[r + 1];
    double *w = data + s.off + (int64_t)q * (N + 2 * kMaxHalf);
    for (int k = 0; k < N + 2 * kMaxHalf; ++k) w[k] = 0.0;
    for (int r = 0; r < N; ++r) add_dr_row(s, ext, r, z[r], w);
}

// One (pass, operator) of an iterated plan, with its lines' end values at
// units ubase .. ubase + nunits - 1 (unit = field * nlines + line, two values
// each: the left and right end-node values, or end values).
struct IterOp {
    int pass, o;
    int nbr_m, nbr_p;            // the same pass and operator on the neighbouring blocks
    int64_t ubase;
    int nunits;
    int N, c, Npad;
    int64_t wofs;                // end weights (4 x (N + 2 kMaxHalf) doubles)
    int64_t gofs;                // influence vectors g-, g+ in the FP64 tables ([2][Npad])
    double hinv;
};

// Per line: iterate-0 end-node values (ends0) and the xf values (endsf).
template <typename T>
__global__ void k_end_values(const IterOp *__restrict__ ops, const PassDesc *__restrict__ passes,
                             const double *__restrict__ weights, const T *__restrict__ in, T *__restrict__ ends0,
                             T *__restrict__ endsf) {
    const IterOp op = ops[blockIdx.y];
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= op.nunits) return;
    const PassDesc &pd = passes[op.pass];
    const int f = u / pd.nlines;
    const int line = u - f * pd.nlines;
    const int lu = line % pd.nu, lv = line / pd.nu;
    const T *src = in + pd.in_base + (int64_t)(pd.field0 + f) * pd.in_fstride + (int64_t)lv * pd.sv +
                   (int64_t)lu * pd.su;
    const int N = op.N;
    const int R = kMaxHalf;
    const int j0 = -min(R, pd.ng), j1 = N + min(R, pd.ng);   // stored nodes; weights beyond are zero
    const double *w = weights + op.wofs;
    const int W = N + 2 * R;
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int j = j0; j < j1; ++j) {
        const T v = src[(int64_t)j * pd.sd];
        s0 += (T)w[j + R] * v;
        s1 += (T)w[W + j + R] * v;
        s2 += (T)w[2 * W + j + R] * v;
        s3 += (T)w[3 * W + j + R] * v;
    }
    const T h = (T)op.hinv;
    const int64_t e = 2 * (op.ubase + u);
    ends0[e] = h * s0;
    ends0[e + 1] = h * s1;
    endsf[e] = h * s2;
    endsf[e + 1] = h * s3;
}

// gather = 0: next = the end-node values of the next iterate; gather = 1:
// next = each line's end values for the iterate after prev (left: the left
// neighbour's value at N - c, right: the right neighbour's at c - 1).
template <typename T>
__global__ void k_iter_ends(const IterOp *__restrict__ ops, const double *__restrict__ tabs64,
                            const T *__restrict__ endsf, const T *__restrict__ prev, T *__restrict__ next, int gather) {
    const IterOp op = ops[blockIdx.y];
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= op.nunits) return;
    const int64_t e = 2 * (op.ubase + u);
    const T em = prev[2 * (ops[op.nbr_m].ubase + u) + 1];
    const T ep = prev[2 * (ops[op.nbr_p].ubase + u)];
    if (gather) {
        next[e] = em;
        next[e + 1] = ep;
        return;
    }
    const double *gm = tabs64 + op.gofs, *gp = gm + op.Npad;
    const int jl = op.c - 1, jr = op.N - op.c;
    next[e] = endsf[e] + (T)gm[jl] * em + (T)gp[jl] * ep;
    next[e + 1] = endsf[e + 1] + (T)gm[jr] * em + (T)gp[jr] * ep;
}

size_t end_weight_spec_size() { return sizeof(EndWeightSpec); }
size_t iter_op_size() { return sizeof(IterOp); }

void fill_end_weight_spec(void *dst, int N, int c, const Scheme &blk, const Scheme &it, int64_t off) {
    EndWeightSpec s;
    s.N = N;
    s.c = c;
    s.d = blk.d;
    s.alpha = blk.lhs[kMaxNL + 1];
    for (int m = 0; m < 2 * kMaxHalf + 1; ++m) {
        s.a[m] = blk.rhs[m];
        s.cl[m] = blk.cl[0][m];
        s.ce[m] = it.cl[0][m];
    }
    s.cl_d0 = it.cl_d0;
    s.cl_up = it.cl_up;
    s.off = off;
    *reinterpret_cast<EndWeightSpec *>(dst) = s;
}

void fill_iter_op(void *dst, int pass, int o, int nbr_m, int nbr_p, int64_t ubase, int nunits, int N, int c, int Npad,
                  int64_t wofs, int64_t gofs, double hinv) {
    IterOp r;
    r.pass = pass;
    r.o = o;
    r.nbr_m = nbr_m;
    r.nbr_p = nbr_p;
    r.ubase = ubase;
    r.nunits = nunits;
    r.N = N;
    r.c = c;
    r.Npad = Npad;
    r.wofs = wofs;
    r.gofs = gofs;
    r.hinv = hinv;
    *reinterpret_cast<IterOp *>(dst) = r;
}

hipError_t launch_end_weights(int ntab, const void *specs, double *data, double *scratch, int stride, hipStream_t st) {
    hipLaunchKernelGGL(k_end_weights, dim3((4 * ntab + 63) / 64), dim3(64), 0, st, ntab,
                       (const EndWeightSpec *)specs, data, scratch, stride);
    return hipGetLastError();
}

hipError_t launch_end_values(int f32, int nops, int max_units, const void *ops, const PassDesc *passes,
                             const double *weights, const void *in, void *ends0, void *endsf, hipStream_t st) {
    const dim3 grid((max_units + 255) / 256, nops);
    if (f32)
        hipLaunchKernelGGL(k_end_values<float>, grid, dim3(256), 0, st, (const IterOp *)ops, passes, weights,
                           (const float *)in, (float *)ends0, (float *)endsf);
    else
        hipLaunchKernelGGL(k_end_values<double>, grid, dim3(256), 0, st, (const IterOp *)ops, passes, weights,
                           (const double *)in, (double *)ends0, (double *)endsf);
    return hipGetLastError();
}

hipError_t launch_iter_ends(int f32, int nops, int max_units, const void *ops, const double *tabs64, const void *endsf,
                            const void *prev, void *next, int gather, hipStream_t st) {
    const dim3 grid((max_units + 255) / 256, nops);
    if (f32)
        hipLaunchKernelGGL(k_iter_ends<float>, grid, dim3(256), 0, st, (const IterOp *)ops, tabs64,
                           (const float *)endsf, (const float *)prev, (float *)next, gather);
    else
        hipLaunchKernelGGL(k_iter_ends<double>, grid, dim3(256), 0, st, (const IterOp *)ops, tabs64,
                           (const double *)endsf, (const double *)prev, (double *)next, gather);
    return hipGetLastError();
}

}  // namespace cfd
