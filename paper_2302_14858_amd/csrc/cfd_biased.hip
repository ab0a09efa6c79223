// Biased (upwind) compact first derivatives on the lines of mesh blocks
// (arXiv 2302.14858, Sec. ssec:domdec_drp).
//
// Left-biased rows: alpha x_{k-1} + x_k = sum_m a_m f_{k+m} (k > k*_-), with
// the closure row x_{k*_-} + alpha x_{k*_- + 1} = sum_m c_m f_{k*_- + m}
// (Eq. closure_left_X).  The right-biased operator is the mirror image:
// x_k + alpha x_{k+1} = -sum_m a_{-m} f_{k+m} (k < k*_+), closure row
// alpha x_{k*_+ - 1} + x_{k*_+} = -sum_m c_{-m} f_{k*_+ + m}.  Each system is
// bidiagonal apart from its closure row, so the two rows at the closed end
// are solved together and the rest is one recurrence away from that end.
// On periodic lines every row is an interior row with indices taken modulo N;
// the cyclic recurrence is closed by its wrap value
//   x^L_{N-1} = sum_j (-alpha)^(N-1-j) r^L_j / (1 - (-alpha)^N),
//   x^R_0     = sum_j (-alpha)^j r^R_j       / (1 - (-alpha)^N),
// both accumulated in one forward pre-sweep.
//
// Upwind operator (Eq. biasderapproxadv, with c the velocity field sampled on
// the grid): c d f = min(c, 0) D[right] f + max(c, 0) D[left] f.
//
// One lane per line, 64 lines per wave, four independent waves per
// workgroup.  Lanes run along the contiguous direction of the block for y
// and z lines, so every load and store of a wave is one coalesced access.
// A lane keeps a register window of 2 HB + 3 samples (offsets -(HB+1) ..
// HB+1 around the current row) and slides it one node per row.  The right-
// biased sweep runs first (from k*_+ down) and leaves min(c,0) D[right] f in
// the output; the left-biased sweep (from k*_- up) adds max(c,0) D[left] f.
#include <hip/hip_runtime.h>

#include "cfd_internal.h"

namespace cfd {
namespace {

template <typename T>
struct BLine {
    const T *f;
    int64_t sd;
    int N, ng, periodic;
    __device__ __forceinline__ T ld(int j) const {
        if (periodic) {
            j %= N;
            if (j < 0) j += N;
            return f[(int64_t)j * sd];
        }
        return (j >= -ng && j < N + ng) ? f[(int64_t)j * sd] : T(0);
    }
};

template <typename T, int HB>
struct BCoef {
    T alpha, inv_det;
    T a[2 * HB + 1];   // a_{-HB..HB}
    T c[2 * HB + 2];   // c_{-HB..HB+1}
};

// window index of offset m: HB + 1 + m
template <typename T, int HB>
__device__ __forceinline__ T left_interior(const BCoef<T, HB> &q, const T *w) {
    T r = 0;
#pragma unroll
    for (int m = -HB; m <= HB; ++m) r += q.a[m + HB] * w[HB + 1 + m];
    return r;
}
template <typename T, int HB>
__device__ __forceinline__ T left_closure(const BCoef<T, HB> &q, const T *w) {
    T r = 0;
#pragma unroll
    for (int m = -HB; m <= HB + 1; ++m) r += q.c[m + HB] * w[HB + 1 + m];
    return r;
}
template <typename T, int HB>
__device__ __forceinline__ T right_interior(const BCoef<T, HB> &q, const T *w) {
    T r = 0;
#pragma unroll
    for (int m = -HB; m <= HB; ++m) r -= q.a[m + HB] * w[HB + 1 - m];
    return r;
}
template <typename T, int HB>
__device__ __forceinline__ T right_closure(const BCoef<T, HB> &q, const T *w) {
    T r = 0;
#pragma unroll
    for (int m = -HB; m <= HB + 1; ++m) r -= q.c[m + HB] * w[HB + 1 - m];
    return r;
}

template <typename T, int HB>
__global__ __launch_bounds__(256) void k_biased(const BiasItem *__restrict__ items, int nitems,
                                                const BiasPass *__restrict__ passes, const T *__restrict__ coefs,
                                                const T *__restrict__ in, T *__restrict__ out) {
    constexpr int W = 2 * HB + 3;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int it = blockIdx.x * 4 + wv;
    if (it >= nitems) return;
    const BiasItem item = items[it];
    const BiasPass ps = passes[item.pass];
    const int line = item.line0 + lane;
    if (line >= ps.nlines) return;
    const int u = line % ps.nu, v = line / ps.nu;

    BCoef<T, HB> q;
    {
        const T *rec = coefs + (int64_t)ps.tab * kBiasRec;
        q.alpha = rec[0];
        q.inv_det = rec[24];
#pragma unroll
        for (int m = -HB; m <= HB; ++m) q.a[m + HB] = rec[1 + kBiasHalf + m];
#pragma unroll
        for (int m = -HB; m <= HB + 1; ++m) q.c[m + HB] = rec[12 + kBiasHalf + m];
    }
    const int N = ps.N;
    BLine<T> L{in + ps.in_base + (int64_t)item.field * ps.in_fstride + (int64_t)u * ps.su + (int64_t)v * ps.sv,
               ps.sd, N, ps.ng, ps.periodic};
    const T *vel = (ps.mode == 0) ? in + ps.vel_base + (int64_t)u * ps.su + (int64_t)v * ps.sv : nullptr;
    T *o = out + ps.out_base + (int64_t)item.field * ps.out_fstride + (int64_t)u * ps.osu + (int64_t)v * ps.osv;
    const int64_t osd = ps.osd;
    const T hinv = (T)ps.hinv;
    const T alpha = q.alpha;
    T w[W];

    T xl_wrap = 0, xr_wrap = 0;
    if (ps.periodic) {
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(i - (HB + 1));
        T sl = 0, sr = 0, pw = 1;
        for (int k = 0; k < N; ++k) {
            if (ps.mode <= 0) sl = sl * (-alpha) + left_interior<T, HB>(q, w);
            if (ps.mode >= 0) {
                sr += pw * right_interior<T, HB>(q, w);
                pw *= -alpha;
            }
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(k + 1 + HB + 1);
        }
        xl_wrap = sl * (T)ps.wrap;
        xr_wrap = sr * (T)ps.wrap;
    }

    // right-biased sweep, k = N-1 .. 0
    if (ps.mode >= 0) {
        auto emit = [&](int k, T x) {
            T val = hinv * x;
            if (ps.mode == 0) val = fmin(vel[(int64_t)k * ps.sd], (T)0) * val;
            o[(int64_t)k * osd] = val;
        };
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(N - 1 - (HB + 1) + i);
        int k = N - 1;
        T xn = xr_wrap;
        if (!ps.periodic) {
            const T rb = right_closure<T, HB>(q, w);
#pragma unroll
            for (int i = W - 1; i > 0; --i) w[i] = w[i - 1];
            w[0] = L.ld(N - 2 - (HB + 1));
            const T r = right_interior<T, HB>(q, w);
            const T xe = (rb - alpha * r) * q.inv_det;
            xn = r - alpha * xe;
            emit(N - 1, xe);
            emit(N - 2, xn);
#pragma unroll
            for (int i = W - 1; i > 0; --i) w[i] = w[i - 1];
            w[0] = L.ld(N - 3 - (HB + 1));
            k = N - 3;
        }
        for (; k >= 0; --k) {
            const T x = right_interior<T, HB>(q, w) - alpha * xn;
            emit(k, x);
            xn = x;
#pragma unroll
            for (int i = W - 1; i > 0; --i) w[i] = w[i - 1];
            w[0] = L.ld(k - 1 - (HB + 1));
        }
    }

    // left-biased sweep, k = 0 .. N-1
    if (ps.mode <= 0) {
        auto emit = [&](int k, T x) {
            T val = hinv * x;
            if (ps.mode == 0) val = o[(int64_t)k * osd] + fmax(vel[(int64_t)k * ps.sd], (T)0) * val;
            o[(int64_t)k * osd] = val;
        };
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(i - (HB + 1));
        int k = 0;
        T xp = xl_wrap;
        if (!ps.periodic) {
            const T rb = left_closure<T, HB>(q, w);
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(1 + HB + 1);
            const T r = left_interior<T, HB>(q, w);
            const T x0 = (rb - alpha * r) * q.inv_det;
            xp = r - alpha * x0;
            emit(0, x0);
            emit(1, xp);
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(2 + HB + 1);
            k = 2;
        }
        for (; k < N; ++k) {
            const T x = left_interior<T, HB>(q, w) - alpha * xp;
            emit(k, x);
            xp = x;
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(k + 1 + HB + 1);
        }
    }
}

template <typename T>
const void *biased_fn(int hb) {
    switch (hb) {
        case 2: return (const void *)k_biased<T, 2>;
        case 3: return (const void *)k_biased<T, 3>;
        case 4: return (const void *)k_biased<T, 4>;
        case 5: return (const void *)k_biased<T, 5>;
        default: return nullptr;
    }
}

}  // namespace

bool biased_supported(int hb) { return hb >= 2 && hb <= 5; }

hipError_t launch_biased(int f32, int hb, const BiasItem *items, int nitems, const BiasPass *passes,
                         const void *coefs, const void *in, void *out, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const int grid = (nitems + 3) / 4;
    if (f32) {
        const void *fn = biased_fn<float>(hb);
        if (!fn) return hipErrorInvalidValue;
        hipLaunchKernelGGL(((void (*)(const BiasItem *, int, const BiasPass *, const float *, const float *,
                                      float *))fn),
                           dim3(grid), dim3(256), 0, st, items, nitems, passes, (const float *)coefs,
                           (const float *)in, (float *)out);
    } else {
        const void *fn = biased_fn<double>(hb);
        if (!fn) return hipErrorInvalidValue;
        hipLaunchKernelGGL(((void (*)(const BiasItem *, int, const BiasPass *, const double *, const double *,
                                      double *))fn),
                           dim3(grid), dim3(256), 0, st, items, nitems, passes, (const double *)coefs,
                           (const double *)in, (double *)out);
    }
    return hipGetLastError();
}

}  // namespace cfd
