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
// W schemes (Tab. ccuw_deg_one_col) add w2 s_k to every interior row's right
// side (-w2 s_k for the right bias), s the embedded second derivative another
// launch left in the plan scratch and w2 = a2 h^2; the closure rows take none.
// U schemes (Tab. ucd_slow) read s, the sampled f'', from an input field and
// add it on every row, the closure row with its own weight w2c.
//
// Partitioned kernel (lines of up to 64 nodes): one lane per line, 64 lines
// per wave; a line is cut into P = 1, 2 or 4 partitions of at most L = 8, 12
// or 16 rows (the fewest partitions with at most 12 rows where possible),
// one wave each, so a workgroup of four waves holds 4 / P groups of 64
// lines.  A wave issues every load of its partition (its rows and the
// stencil halo) before any arithmetic and keeps them in registers.  Each
// bias is solved locally with a zero value entering the partition (the
// closure rows where the partition holds them); the exact solution is the
// local one plus (-alpha)^distance times the true value entering it.  The
// waves exchange their local end values through LDS and each walks the
// chain of partitions before it (around the line on periodic lines, closed
// by 1 / (1 - (-alpha)^N)) to get its entering values.  Lanes run along the
// contiguous direction of the block for y and z lines, so each load and
// store of a wave is one coalesced access; x lines are staged through an LDS
// tile filled and drained with contiguous accesses along the rows.
//
// Sweep kernel (longer lines): one lane per line, a register window of
// 2 HB + 3 samples slid one node per row; the right-biased sweep leaves
// min(c,0) D[right] f in the output, the left-biased sweep adds the rest.
#include <hip/hip_runtime.h>

#include <algorithm>

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
__device__ __forceinline__ void load_coef(BCoef<T, HB> &q, const T *rec) {
    q.alpha = rec[0];
    q.inv_det = rec[24];
#pragma unroll
    for (int m = -HB; m <= HB; ++m) q.a[m + HB] = rec[1 + kBiasHalf + m];
#pragma unroll
    for (int m = -HB; m <= HB + 1; ++m) q.c[m + HB] = rec[12 + kBiasHalf + m];
}

// Walk of a thread over the elements e = threadIdx.x, + 256, ... of a
// [lines][cols] tile (cols <= 256) in row-major order, with the (u, v) position of its line
// kept up to date, so the fill and drain loops divide only once.
struct TileWalk {
    int l, j, dq, dr, cols;   // row (line of the workgroup), column, row / column step
    int ln, uu, vv;           // line index in the pass, its u and v
    __device__ __forceinline__ TileWalk(int t, int cols_, int line0, int nu) : cols(cols_) {
        l = t / cols;
        j = t - l * cols;
        dq = 256 / cols;
        dr = 256 - dq * cols;
        ln = line0 + l;
        uu = ln % nu;
        vv = ln / nu;
    }
    __device__ __forceinline__ void next(int nu) {
        int dl = dq;
        j += dr;
        if (j >= cols) {
            j -= cols;
            ++dl;
        }
        l += dl;
        ln += dl;
        uu += dl;
        while (uu >= nu) {
            uu -= nu;
            ++vv;
        }
    }
};

// LDS: exchange area [4 waves][2][64], then (x lines) the tile of the
// workgroup's lines, [4/P groups x 64 lines][pitch].
// Iterated closures (Eq. iter_left_X and its mirror; ev given): every row of
// a closure line takes the interior scheme, and the solution entering at node
// -1 (left bias) / N (right bias) is ev[2 e] / ev[2 e + 1] of the line's
// entry e = ev_base + field * nlines + line, instead of the closure rows.
// ends (if given) receives, unscaled (before h^-1), the left-biased solution
// at node N - 1 and the right-biased one at node 0 of every line, the values
// the neighbours' next iterate enters with.
template <typename T, int HB, int L, bool XDIR>
__global__ __launch_bounds__(256) void k_biased_part(const BiasItem *__restrict__ items,
                                                     const BiasPass *__restrict__ passes,
                                                     const T *__restrict__ coefs, const T *__restrict__ in,
                                                     T *__restrict__ out, const T *__restrict__ ev,
                                                     T *__restrict__ ends) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int W = L + 2 * HB + 2;   // f[i] = node k0 - HB - 1 + i
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const BiasItem item = items[blockIdx.x];
    if (item.pass < 0) return;   // padding of the XCD-interleaved order (whole workgroup)
    const BiasPass ps = passes[item.pass];
    const int P = item.P, G = 4 / P;
    const int g = wv / P, p = wv - g * P;
    const int N = ps.N, Lr = (N + P - 1) / P;
    const int k0 = p * Lr;
    const int nrows = min(Lr, N - k0);   // >= 2: the host picks P so that every partition has 2 rows
    const int line = item.line0 + 64 * g + lane;
    const bool active = line < ps.nlines;
    const int u = active ? line % ps.nu : 0, v = active ? line / ps.nu : 0;
    const int64_t fbase = ps.in_base + (int64_t)item.field * ps.in_fstride;
    const int64_t obase = ps.out_base + (int64_t)item.field * ps.out_fstride;
    T *exch = (T *)smem;
    T *tile = exch + 4 * 2 * 64;
    const bool periodic = ps.periodic;
    const bool iter = ev != nullptr && !periodic;
    const bool closureL = !periodic && p == 0 && !iter;
    const bool closureR = !periodic && p == P - 1 && !iter;
    const int64_t eix = 2 * (ps.ev_base + (int64_t)item.field * ps.nlines + line);   // this line's end entries
    const int mode = ps.mode;
    const T *rec = coefs + (int64_t)ps.tab * kBiasRec;
    BCoef<T, HB> q;
    load_coef<T, HB>(q, rec);
    const T alpha = q.alpha;

    // ---- partition rows and halo into registers
    T f[W];
    int vp = N | 1;   // x lines: pitch of the velocity / output tile
    if (XDIR) {
        int t0, Tn;
        if (periodic) {
            t0 = 0;
            Tn = N;
        } else {
            const int e = min(ps.ng, HB + 1);
            t0 = -e;
            Tn = N + 2 * e;
        }
        const int tp = Tn | 1;
        const int nl = 64 * G;
        // consecutive threads take consecutive nodes of the workgroup's rows
        for (TileWalk w(threadIdx.x, Tn, item.line0, ps.nu); w.l < nl; w.next(ps.nu)) {
            T val = 0;
            if (w.ln < ps.nlines) val = in[fbase + (int64_t)w.uu * ps.su + (int64_t)w.vv * ps.sv + (t0 + w.j)];
            tile[w.l * tp + w.j] = val;
        }
        __syncthreads();
        const T *row = tile + (64 * g + lane) * tp;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            int j = k0 - HB - 1 + i;
            if (periodic) {
                j %= N;
                if (j < 0) j += N;
                f[i] = row[j];
            } else {
                f[i] = (j >= t0 && j < t0 + Tn) ? row[j - t0] : T(0);
            }
        }
        __syncthreads();   // the tile is reused for the velocity and the output
        if (mode == 0) {
            for (TileWalk w(threadIdx.x, N, item.line0, ps.nu); w.l < nl; w.next(ps.nu)) {
                T val = 0;
                if (w.ln < ps.nlines) val = in[ps.vel_base + (int64_t)w.uu * ps.su + (int64_t)w.vv * ps.sv + w.j];
                tile[w.l * vp + w.j] = val;
            }
        }
    } else {
        BLine<T> Lf{in + fbase + (int64_t)u * ps.su + (int64_t)v * ps.sv, ps.sd, N, ps.ng, periodic};
#pragma unroll
        for (int i = 0; i < W; ++i) f[i] = active ? Lf.ld(k0 - HB - 1 + i) : T(0);
    }

    // ---- right-hand sides (closure rows where this partition holds them)
    T rl[L], rr[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        rl[i] = (closureL && i == 0) ? left_closure<T, HB>(q, f + i) : left_interior<T, HB>(q, f + i);
        rr[i] = (closureR && i == nrows - 1) ? right_closure<T, HB>(q, f + i) : right_interior<T, HB>(q, f + i);
    }
    if ((ps.s2 || ps.s2_in) && active) {   // W, U: the second-derivative term of each row
        const T *s2 = (ps.s2_in ? in : (const T *)ps.s2) + ps.s2_base + (int64_t)item.field * ps.s2f +
                      (int64_t)u * ps.s2u + (int64_t)v * ps.s2v;
        const T w2 = (T)ps.w2, w2c = (T)ps.w2c;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if (i < nrows) {
                const T e = s2[(int64_t)(k0 + i) * ps.s2d];
                rl[i] += ((closureL && i == 0) ? w2c : w2) * e;
                rr[i] -= ((closureR && i == nrows - 1) ? w2c : w2) * e;
            }
        }
    }

    // ---- local solves with zero entering values
    T xl_last = 0, xr_first = 0;
    const bool left = mode <= 0 || mode == 2;   // -1 left, 0 upwind, 2 symmetrised: the left-biased solve
    if (left) {
        T xp = 0;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const T x = (closureL && i == 0) ? (rl[0] - alpha * rl[1]) * q.inv_det : rl[i] - alpha * xp;
            rl[i] = x;
            xp = x;
            if (i == nrows - 1) xl_last = x;
        }
    }
    if (mode >= 0) {
        T xn = 0;
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            T x;
            if (i >= nrows) x = 0;
            else if (closureR && i == nrows - 1) x = (rr[i] - alpha * (i > 0 ? rr[i > 0 ? i - 1 : 0] : T(0))) * q.inv_det;
            else x = rr[i] - alpha * xn;
            rr[i] = x;
            xn = x;
        }
        xr_first = rr[0];
    }
    // velocity of y/z lines: loaded here so that the loads overlap the exchange
    T c[L];
    if (!XDIR && mode == 0) {
        const T *vl = in + ps.vel_base + (int64_t)u * ps.su + (int64_t)v * ps.sv;
#pragma unroll
        for (int i = 0; i < L; ++i) c[i] = (active && i < nrows) ? vl[(int64_t)(k0 + i) * ps.sd] : T(0);
    }
    exch[(wv * 2 + 0) * 64 + lane] = xl_last;
    exch[(wv * 2 + 1) * 64 + lane] = xr_first;
    __syncthreads();

    // ---- true values entering the partition
    const T *pw = rec + kBiasPow;   // (-alpha)^n
    T X = 0, Y = 0;
    if (iter && active) {   // the values entering the line, from the neighbours' previous iterate
        X = ev[eix];
        Y = ev[eix + 1];
    }
    if (left) {
        if (periodic) {
            T s = 0;
            for (int qq = 0; qq < P; ++qq) {
                const int k1 = min(qq * Lr + Lr, N) - 1;
                s += pw[N - 1 - k1] * exch[((g * P + qq) * 2 + 0) * 64 + lane];
            }
            X = s * (T)ps.wrap;
        }
        for (int qq = 0; qq < p; ++qq) X = exch[((g * P + qq) * 2 + 0) * 64 + lane] + pw[min(Lr, N - qq * Lr)] * X;
    }
    if (mode >= 0) {
        if (periodic) {
            T s = 0;
            for (int qq = 0; qq < P; ++qq) s += pw[qq * Lr] * exch[((g * P + qq) * 2 + 1) * 64 + lane];
            Y = s * (T)ps.wrap;
        }
        for (int qq = P - 1; qq > p; --qq) Y = exch[((g * P + qq) * 2 + 1) * 64 + lane] + pw[min(Lr, N - qq * Lr)] * Y;
    }

    // ---- the line's end values for the neighbours' next iterate (unscaled)
    if (ends && active && !periodic) {
        if (left && p == P - 1) ends[eix] = rl[nrows - 1] + pw[nrows] * X;
        if (mode >= 0 && p == 0) ends[eix + 1] = rr[0] + pw[nrows] * Y;
    }

    // ---- corrected values, combined and stored
    const T hinv = (T)ps.hinv;
    T *tl = tile + (64 * g + lane) * vp;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        if (i < nrows) {
            T val;
            if (mode < 0) {
                val = hinv * (rl[i] + pw[i + 1] * X);
            } else if (mode == 1) {
                val = hinv * (rr[i] + pw[nrows - i] * Y);
            } else if (mode == 2) {
                val = T(0.5) * (hinv * (rl[i] + pw[i + 1] * X) + hinv * (rr[i] + pw[nrows - i] * Y));
            } else {
                const T cv = XDIR ? tl[k0 + i] : c[i];
                const T xL = rl[i] + pw[i + 1] * X;
                const T xR = rr[i] + pw[nrows - i] * Y;
                val = fmin(cv, (T)0) * (hinv * xR) + fmax(cv, (T)0) * (hinv * xL);
            }
            if (XDIR) tl[k0 + i] = val;
            else if (active) out[obase + (int64_t)u * ps.osu + (int64_t)v * ps.osv + (int64_t)(k0 + i) * ps.osd] = val;
        }
    }
    if (XDIR) {
        __syncthreads();
        const int nl = 64 * G;
        for (TileWalk w(threadIdx.x, N, item.line0, ps.nu); w.l < nl; w.next(ps.nu))
            if (w.ln < ps.nlines) out[obase + (int64_t)w.uu * ps.osu + (int64_t)w.vv * ps.osv + w.j] = tile[w.l * vp + w.j];
    }
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
    // W, U: the second-derivative term at node k, interior rows (e2) and closure row (e2c)
    const T *s2 = (ps.s2 || ps.s2_in) ? (ps.s2_in ? in : (const T *)ps.s2) + ps.s2_base +
                                            (int64_t)item.field * ps.s2f + (int64_t)u * ps.s2u +
                                            (int64_t)v * ps.s2v
                                      : nullptr;
    const T w2 = (T)ps.w2, w2c = (T)ps.w2c;
    auto e2 = [&](int k) -> T { return s2 ? w2 * s2[(int64_t)k * ps.s2d] : T(0); };
    auto e2c = [&](int k) -> T { return s2 ? w2c * s2[(int64_t)k * ps.s2d] : T(0); };

    T xl_wrap = 0, xr_wrap = 0;
    if (ps.periodic) {
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(i - (HB + 1));
        T sl = 0, sr = 0, pw = 1;
        for (int k = 0; k < N; ++k) {
            if (ps.mode <= 0 || ps.mode == 2) sl = sl * (-alpha) + (left_interior<T, HB>(q, w) + e2(k));
            if (ps.mode >= 0) {
                sr += pw * (right_interior<T, HB>(q, w) - e2(k));
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
            if (ps.mode == 2) val = T(0.5) * val;
            o[(int64_t)k * osd] = val;
        };
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(N - 1 - (HB + 1) + i);
        int k = N - 1;
        T xn = xr_wrap;
        if (!ps.periodic) {
            const T rb = right_closure<T, HB>(q, w) - e2c(N - 1);
#pragma unroll
            for (int i = W - 1; i > 0; --i) w[i] = w[i - 1];
            w[0] = L.ld(N - 2 - (HB + 1));
            const T r = right_interior<T, HB>(q, w) - e2(N - 2);
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
            const T x = (right_interior<T, HB>(q, w) - e2(k)) - alpha * xn;
            emit(k, x);
            xn = x;
#pragma unroll
            for (int i = W - 1; i > 0; --i) w[i] = w[i - 1];
            w[0] = L.ld(k - 1 - (HB + 1));
        }
    }

    // left-biased sweep, k = 0 .. N-1
    if (ps.mode <= 0 || ps.mode == 2) {
        auto emit = [&](int k, T x) {
            T val = hinv * x;
            if (ps.mode == 0) val = o[(int64_t)k * osd] + fmax(vel[(int64_t)k * ps.sd], (T)0) * val;
            if (ps.mode == 2) val = o[(int64_t)k * osd] + T(0.5) * val;
            o[(int64_t)k * osd] = val;
        };
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = L.ld(i - (HB + 1));
        int k = 0;
        T xp = xl_wrap;
        if (!ps.periodic) {
            const T rb = left_closure<T, HB>(q, w) + e2c(0);
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(1 + HB + 1);
            const T r = left_interior<T, HB>(q, w) + e2(1);
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
            const T x = (left_interior<T, HB>(q, w) + e2(k)) - alpha * xp;
            emit(k, x);
            xp = x;
#pragma unroll
            for (int i = 0; i < W - 1; ++i) w[i] = w[i + 1];
            w[W - 1] = L.ld(k + 1 + HB + 1);
        }
    }
}

template <typename T>
const void *sweep_fn(int hb) {
    switch (hb) {
        case 2: return (const void *)k_biased<T, 2>;
        case 3: return (const void *)k_biased<T, 3>;
        case 4: return (const void *)k_biased<T, 4>;
        case 5: return (const void *)k_biased<T, 5>;
        default: return nullptr;
    }
}

template <typename T, int HB>
const void *part_fn_hb(int L, int xdir) {
    if (L == 8) return xdir ? (const void *)k_biased_part<T, HB, 8, true> : (const void *)k_biased_part<T, HB, 8, false>;
    if (L == 12) return xdir ? (const void *)k_biased_part<T, HB, 12, true> : (const void *)k_biased_part<T, HB, 12, false>;
    if (L == 16) return xdir ? (const void *)k_biased_part<T, HB, 16, true> : (const void *)k_biased_part<T, HB, 16, false>;
    return nullptr;
}

template <typename T>
const void *part_fn(int hb, int L, int xdir) {
    switch (hb) {
        case 2: return part_fn_hb<T, 2>(L, xdir);
        case 3: return part_fn_hb<T, 3>(L, xdir);
        case 4: return part_fn_hb<T, 4>(L, xdir);
        case 5: return part_fn_hb<T, 5>(L, xdir);
        default: return nullptr;
    }
}

}  // namespace

bool biased_supported(int hb) { return hb >= 2 && hb <= 5; }

size_t biased_lds(int f32, int hb, int L, int xdir, int P, int N) {
    if (L == 0) return 0;
    const size_t es = f32 ? 4 : 8;
    size_t b = 4 * 2 * 64 * es;
    if (xdir) {
        const int e = hb + 1;   // at most this many ghost nodes per side are staged
        const int tp = (N + 2 * e) | 1;
        b += (size_t)(4 / P) * 64 * (size_t)std::max(tp, N | 1) * es;
    }
    return b;
}

// End values of the next iterate: for every biased pass (rec = ev base of
// the pass, of its left neighbour along the lines, of its right neighbour,
// entries), entry e takes the left neighbour's left-biased last value and the
// right neighbour's right-biased first value of the same field and line.
template <typename T>
__global__ void k_bias_gather(const int64_t *__restrict__ recs, const T *__restrict__ ends, T *__restrict__ ev) {
    const int64_t *r = recs + 4 * blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r[3]) return;
    ev[2 * (r[0] + e)] = ends[2 * (r[1] + e)];
    ev[2 * (r[0] + e) + 1] = ends[2 * (r[2] + e) + 1];
}

hipError_t launch_bias_gather(int f32, int npass, int64_t max_entries, const int64_t *recs, const void *ends, void *ev,
                              hipStream_t st) {
    if (npass == 0 || max_entries == 0) return hipSuccess;
    const dim3 grid((unsigned)((max_entries + 255) / 256), (unsigned)npass);
    if (f32)
        hipLaunchKernelGGL(k_bias_gather<float>, grid, dim3(256), 0, st, recs, (const float *)ends, (float *)ev);
    else
        hipLaunchKernelGGL(k_bias_gather<double>, grid, dim3(256), 0, st, recs, (const double *)ends, (double *)ev);
    return hipGetLastError();
}

hipError_t launch_biased(int f32, int hb, int L, int xdir, size_t lds, const BiasItem *items, int nitems,
                         const BiasPass *passes, const void *coefs, const void *in, void *out, const void *ev,
                         void *ends, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (L == 0) {
        const int grid = (nitems + 3) / 4;
        const void *fn = f32 ? sweep_fn<float>(hb) : sweep_fn<double>(hb);
        if (!fn) return hipErrorInvalidValue;
        if (f32)
            hipLaunchKernelGGL(((void (*)(const BiasItem *, int, const BiasPass *, const float *, const float *,
                                          float *))fn),
                               dim3(grid), dim3(256), 0, st, items, nitems, passes, (const float *)coefs,
                               (const float *)in, (float *)out);
        else
            hipLaunchKernelGGL(((void (*)(const BiasItem *, int, const BiasPass *, const double *, const double *,
                                          double *))fn),
                               dim3(grid), dim3(256), 0, st, items, nitems, passes, (const double *)coefs,
                               (const double *)in, (double *)out);
        return hipGetLastError();
    }
    const void *fn = f32 ? part_fn<float>(hb, L, xdir) : part_fn<double>(hb, L, xdir);
    if (!fn) return hipErrorInvalidValue;
    if (f32)
        hipLaunchKernelGGL(((void (*)(const BiasItem *, const BiasPass *, const float *, const float *, float *,
                                      const float *, float *))fn),
                           dim3(nitems), dim3(256), lds, st, items, passes, (const float *)coefs, (const float *)in,
                           (float *)out, (const float *)ev, (float *)ends);
    else
        hipLaunchKernelGGL(((void (*)(const BiasItem *, const BiasPass *, const double *, const double *, double *,
                                      const double *, double *))fn),
                           dim3(nitems), dim3(256), lds, st, items, passes, (const double *)coefs,
                           (const double *)in, (double *)out, (const double *)ev, (double *)ends);
    return hipGetLastError();
}

}  // namespace cfd
