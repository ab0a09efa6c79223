// Dense mixed-precision operator for periodic lines (gfx950).
//
// On a periodic line the compact operator is the circulant matrix
// D = h^-d A^-1 B (the periodic D of Sec. 2.2, formed explicitly as the paper
// remarks one may do with the inverse matrix, Sec. 2.6).  This path:
//   * forms A^-1 B and A^-1 in FP64 on the GPU (dense Gauss-Jordan on
//     [A | B | I], k_dense_form) and keeps row 0 of each (a circulant matrix
//     is its first row): D[i][j] = m[(j - i) mod N], R[i][j] = rho[(j - i) mod N];
//   * splits m into BF16 hi + lo terms and rho into a BF16 hi term;
//   * per tile of 32 lines: yhat = D_hi f_hi + D_hi f_lo + D_lo f_hi on MFMA
//     (v_mfma_f32_16x16x32_bf16, FP32 accumulation), then one refinement with
//     the FP64 banded residual r = h^-d B f - A yhat and y = yhat + R_hi r_hi
//     accumulated into the same registers.
// Inputs and outputs are FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kDenseLines = 32;        // lines per tile (two 16-wide MFMA column blocks)
constexpr int kDensePitch = 34;        // LDS row pitch of the tile (floats): the 4 row groups of a
                                       // B fragment read fall in distinct banks
constexpr int kDenseMaxN = 256;
constexpr int kDenseExt = 16;          // wrap-around margin of the extended circulant rows

// Layout of one dense table (per scheme and line length), in bytes:
//   double coefs[16]:  b_{-5..5} (interior stencil), alpha_{-2..2}
//   bf16 mhi[N+48], mlo[N+48], rhi[N+48]: extended circulant rows,
//       ext[kDenseExt + k] = row[k mod N] for k in [-16, N+32)
struct DenseTab {
    int N;
    int nl, m;     // band and RHS half-width
    int pad;
    int64_t off;   // byte offset of the table
};

__device__ __forceinline__ int wrapN(int k, int N) {
    if (k < 0) k += N;
    if (k >= N) k -= N;
    return k;
}

// ---------------------------------------------------------------------------
// Formation, FP64: one workgroup per table.  M = [A | B | I] (N x 3N) in the
// scratch; Gauss-Jordan with partial pivoting leaves A^-1 B and A^-1 in its right two thirds.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_dense_form(const DenseTab *__restrict__ tabs, const double *__restrict__ coefs_in, double hinv_unused,
             unsigned char *__restrict__ out, double *__restrict__ scratch, int64_t scratch_per,
             int *__restrict__ status) {
    const DenseTab t = tabs[blockIdx.x];
    const int N = t.N, W = 3 * N;
    double *M = scratch + (int64_t)blockIdx.x * scratch_per;
    const double *cf = coefs_in + (int64_t)blockIdx.x * 16;   // b[-5..5] at 0..10, alpha[-2..2] at 11..15
    __shared__ int piv;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    for (int e = threadIdx.x; e < N * W; e += blockDim.x) {
        const int r = e / W, c = e - r * W;
        double v = 0.0;
        if (c < N) {
            const int o = wrapN(c - r, N) <= N / 2 ? wrapN(c - r, N) : wrapN(c - r, N) - N;   // signed offset
            if (o >= -t.nl && o <= t.nl) v = cf[11 + 2 + o];
        } else if (c < 2 * N) {
            const int cc = c - N;
            const int o = wrapN(cc - r, N) <= N / 2 ? wrapN(cc - r, N) : wrapN(cc - r, N) - N;
            if (o >= -t.m && o <= t.m) v = cf[5 + o];
        } else {
            v = (c - 2 * N == r) ? 1.0 : 0.0;
        }
        M[e] = v;
    }
    __syncthreads();
    for (int c = 0; c < N; ++c) {
        if (threadIdx.x == 0) {
            int p = c;
            double best = fabs(M[(int64_t)c * W + c]);
            for (int r = c + 1; r < N; ++r) {
                const double v = fabs(M[(int64_t)r * W + c]);
                if (v > best) { best = v; p = r; }
            }
            if (!(best > 1e-300)) bad = 1;
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != c)
            for (int k = threadIdx.x; k < W; k += blockDim.x) {
                const double a = M[(int64_t)c * W + k];
                M[(int64_t)c * W + k] = M[(int64_t)p * W + k];
                M[(int64_t)p * W + k] = a;
            }
        __syncthreads();
        const double ip = 1.0 / M[(int64_t)c * W + c];
        __syncthreads();
        for (int k = threadIdx.x; k < W; k += blockDim.x) M[(int64_t)c * W + k] *= ip;
        __syncthreads();
        for (int r = 0; r < N; ++r) {
            if (r == c) continue;
            const double f = M[(int64_t)r * W + c];
            if (f == 0.0) continue;
            // columns <= c of the pivot row are already zero or one: touching only k > c keeps
            // M[r][c] (read as f by every thread of this row) unchanged during the update
            for (int k = c + 1 + threadIdx.x; k < W; k += blockDim.x) M[(int64_t)r * W + k] -= f * M[(int64_t)c * W + k];
        }
        __syncthreads();
    }
    // extended circulant rows: D row 0 = (A^-1 B) row 0 (scaled by h^-d at apply
    // time through coefs), R row 0 = (A^-1) row 0
    unsigned char *base = out + t.off;
    double *cfo = reinterpret_cast<double *>(base);
    __bf16 *mhi = reinterpret_cast<__bf16 *>(base + 16 * sizeof(double));
    __bf16 *mlo = mhi + (N + 48);
    __bf16 *rhi = mlo + (N + 48);
    for (int k = threadIdx.x; k < 16; k += blockDim.x) cfo[k] = cf[k];
    for (int j = threadIdx.x; j < N + 48; j += blockDim.x) {
        const int k = wrapN(wrapN(j - kDenseExt, N), N);
        const double d = M[k + N];          // (A^-1 B)[0][k]
        const double r = M[k + 2 * N];      // (A^-1)[0][k]
        const float df = (float)d;
        const __bf16 h = (__bf16)df;
        mhi[j] = h;
        mlo[j] = (__bf16)(float)(d - (double)(float)h);
        rhi[j] = (__bf16)(float)r;
    }
    if (threadIdx.x == 0) status[blockIdx.x] = bad;
}

// ---------------------------------------------------------------------------
// Apply
// ---------------------------------------------------------------------------
struct DenseItem {
    int32_t pass;
    int32_t field;
    int32_t line0;
    int32_t tab;
};

// 8 consecutive circulant entries ext[start .. start + 7] of an extended row: the
// A fragment of lane (q, r) of a 16 x 32 block of D.  start is only 2-byte aligned
// (it moves with r), so five aligned dwords are read and shifted by one element
// where start is odd.
__device__ __forceinline__ bf16x8 circ_frag(const unsigned short *ext, int start) {
    const uint32_t *d = reinterpret_cast<const uint32_t *>(ext) + (start >> 1);
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = d[k];
    const uint32_t sh = (uint32_t)(start & 1) * 2u;   // bytes
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
    bf16x8 v;
    __builtin_memcpy(&v, o, sizeof v);
    return v;
}

// Element offsets of a tile's lines in the input and the output (-1 past the last line).
__device__ __forceinline__ void dense_cols(const DenseItem &wi, const PassDesc *__restrict__ passes, int c,
                                           int64_t *col_in, int64_t *col_out) {
    const PassDesc &pd = passes[wi.pass];
    int64_t a = -1, o = -1;
    if (c < min(kDenseLines, pd.nlines - wi.line0)) {
        const int line = wi.line0 + c;
        const int lu = line % pd.nu, lv = line / pd.nu;
        a = (int64_t)lv * pd.sv + (int64_t)lu * pd.su;
        o = (int64_t)lv * pd.osv + (int64_t)lu * pd.osu;
    }
    col_in[c] = a;
    col_out[c] = o;
}

// Thread <-> tile element maps, element k = 0 .. N/8 - 1 of thread tid:
//  * y/z lines: node g + 8k of line c (c = tid % 32, g = tid / 32): 32 threads
//    read one node of 32 lines that are neighbours in memory;
//  * x lines (nodes consecutive in memory): chunk g + 8k of 32 nodes, node
//    (chunk % (N/32)) * 32 + tid % 32 of line chunk / (N/32).
template <int N, bool XDIR>
__device__ __forceinline__ void dense_elem(int tid, int k, int &i, int &c) {
    const int g = tid >> 5, lane = tid & 31;
    if constexpr (XDIR) {
        constexpr int CPL = N / 32;
        const int chunk = g + 8 * k;
        c = chunk / CPL;
        i = (chunk - c * CPL) * 32 + lane;
    } else {
        c = lane;
        i = g + 8 * k;
    }
}

template <int N, bool XDIR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_dense_apply(const DenseItem *__restrict__ items, int nitems, const PassDesc *__restrict__ passes,
              const DenseTab *__restrict__ tabs, const unsigned char *__restrict__ tabdata,
              const float *__restrict__ in, float *__restrict__ out) {
    constexpr int KT = N / 8;                       // tile elements per thread = rows per residual group
    constexpr int NE = 3 * (N + 48);                // circulant rows (bf16)
    constexpr int EK = (NE + 255) / 256;
    constexpr int NSTRIP = N / 16;                  // 16-row strips of the product
    constexpr int SPW = (NSTRIP + 3) / 4;           // strips per wave
    __shared__ float F[N * kDensePitch];            // input tile, then the result
    __shared__ float Y[N * kDensePitch];            // first approximation yhat, then the residual
    __shared__ __attribute__((aligned(16))) unsigned short Eraw[NE + 8];
    __shared__ int64_t col_in[2][kDenseLines], col_out[2][kDenseLines];   // this tile's and the next one's
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63;
    const int q = l >> 4, r16 = l & 15;
    const int cown = tid & (kDenseLines - 1);
    const int g = tid >> 5;

    // One tile's loads (input and circulant rows) into registers, all in flight at once.
    float pre[KT];
    unsigned short pre_e[EK];
    auto issue_loads = [&](const DenseItem &wi, const int64_t *cin) {
        const PassDesc &pd = passes[wi.pass];
        const float *fbase = in + pd.in_base + (int64_t)(pd.field0 + wi.field) * pd.in_fstride;
        const int64_t sd = pd.sd;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int i, c;
            dense_elem<N, XDIR>(tid, k, i, c);
            // unconditional load (lines past the last one read line 0, then 0 is
            // selected): no branch around it, so all KT loads stay in flight
            const int64_t o = cin[c];
            const float v = fbase[(o >= 0 ? o : 0) + (XDIR ? (int64_t)i : (int64_t)i * sd)];
            pre[k] = o >= 0 ? v : 0.f;
        }
        const unsigned short *ge =
            reinterpret_cast<const unsigned short *>(tabdata + tabs[wi.tab].off + 16 * sizeof(double));
#pragma unroll
        for (int k = 0; k < EK; ++k) {
            const int j = tid + 256 * k;
            pre_e[k] = (j < NE) ? ge[j] : (unsigned short)0;
        }
    };

    if (blockIdx.x < nitems) {
        const DenseItem w0 = items[blockIdx.x];
        if (tid < kDenseLines) dense_cols(w0, passes, tid, col_in[0], col_out[0]);
        __syncthreads();
        issue_loads(w0, col_in[0]);
    }
    int buf = 0;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x, buf ^= 1) {
        const DenseItem wi = items[it];
        const PassDesc &pd = passes[wi.pass];
        const double hinv = pd.hinv[0];
        const double *cf = reinterpret_cast<const double *>(tabdata + tabs[wi.tab].off);

        // 1. the prefetched tile into LDS, F[i][c] = f(node i of line line0 + c);
        // the next tile's loads go out as soon as its line offsets are known
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            int i, c;
            dense_elem<N, XDIR>(tid, k, i, c);
            F[i * kDensePitch + c] = pre[k];
        }
#pragma unroll
        for (int k = 0; k < EK; ++k) {
            const int j = tid + 256 * k;
            if (j < NE) Eraw[j] = pre_e[k];
        }
        const int nxt = it + gridDim.x;
        DenseItem wn{};
        if (nxt < nitems) {
            wn = items[nxt];
            if (tid < kDenseLines) dense_cols(wn, passes, tid, col_in[buf ^ 1], col_out[buf ^ 1]);
        }
        __syncthreads();
        if (nxt < nitems) issue_loads(wn, col_in[buf ^ 1]);

        // 2. yhat = D f on MFMA (v_mfma_f32_16x16x32_bf16): wave w owns strips w, w + 4, ...
        // D = D_hi + D_lo and f = f_hi + f_lo in BF16; the lo * lo term is dropped
        f32x4 acc[SPW][2];
#pragma unroll
        for (int j = 0; j < SPW; ++j) {
            acc[j][0] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[j][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        const unsigned short *mhi = Eraw, *mlo = Eraw + (N + 48), *rhi = Eraw + 2 * (N + 48);
#pragma unroll 1
        for (int k0 = 0; k0 < N; k0 += 32) {
            bf16x8 bh[2], bl[2];
#pragma unroll
            for (int sub = 0; sub < 2; ++sub)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const float v = F[(k0 + 8 * q + t) * kDensePitch + 16 * sub + r16];
                    const __bf16 h = (__bf16)v;
                    bh[sub][t] = h;
                    bl[sub][t] = (__bf16)(v - (float)h);
                }
#pragma unroll
            for (int j = 0; j < SPW; ++j) {
                const int s = w + 4 * j;
                if (s < NSTRIP) {
                    // A fragment: D[16 s + r16][k0 + 8 q + t] = m[(k0 + 8 q + t - 16 s - r16) mod N]
                    const int start = kDenseExt + wrapN(k0 - 16 * s, N) + 8 * q - r16;
                    const bf16x8 ah = circ_frag(mhi, start);
                    const bf16x8 al = circ_frag(mlo, start);
#pragma unroll
                    for (int sub = 0; sub < 2; ++sub) {
                        acc[j][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[sub], acc[j][sub], 0, 0, 0);
                        acc[j][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[sub], acc[j][sub], 0, 0, 0);
                        acc[j][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[sub], acc[j][sub], 0, 0, 0);
                    }
                }
            }
        }
        // the BF16 rows hold A^-1 B; D = h^-d A^-1 B.  yhat into its own tile
        // (C layout: row 16 s + 4 q + t, column 16 sub + r16)
        const float scale = (float)hinv;
#pragma unroll
        for (int j = 0; j < SPW; ++j) {
            const int s = w + 4 * j;
            if (s < NSTRIP)
#pragma unroll
                for (int sub = 0; sub < 2; ++sub)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        acc[j][sub][t] *= scale;
                        Y[(16 * s + 4 * q + t) * kDensePitch + 16 * sub + r16] = acc[j][sub][t];
                    }
        }
        __syncthreads();

        // 3. FP64 residual r = h^-d B f - A yhat on rows g*KT .. g*KT + KT - 1 of column
        // cown, with sliding windows over f (11 nodes) and yhat (5 nodes).  r overwrites
        // yhat in Y: a row is read by another thread only within 2 rows of a group's
        // ends, so those 4 rows wait in registers until every thread is past its reads.
        {
            double cb[11], ca[5];
#pragma unroll
            for (int t = 0; t < 11; ++t) cb[t] = cf[t] * hinv;
#pragma unroll
            for (int t = 0; t < 5; ++t) ca[t] = cf[11 + t];
            const int i0 = g * KT;
            double fw[11], yw[5];
            float edge[4];
#pragma unroll
            for (int t = 0; t < 11; ++t) fw[t] = (double)F[wrapN(i0 - 5 + t, N) * kDensePitch + cown];
#pragma unroll
            for (int t = 0; t < 5; ++t) yw[t] = (double)Y[wrapN(i0 - 2 + t, N) * kDensePitch + cown];
#pragma unroll
            for (int j = 0; j < KT; ++j) {
                double bf = 0.0, ay = 0.0;
#pragma unroll
                for (int t = 0; t < 11; ++t) bf = fma(cb[t], fw[t], bf);
#pragma unroll
                for (int t = 0; t < 5; ++t) ay = fma(ca[t], yw[t], ay);
                const float r = (float)(bf - ay);
                if (j + 1 < KT) {
#pragma unroll
                    for (int t = 0; t < 10; ++t) fw[t] = fw[t + 1];
#pragma unroll
                    for (int t = 0; t < 4; ++t) yw[t] = yw[t + 1];
                    fw[10] = (double)F[wrapN(i0 + j + 6, N) * kDensePitch + cown];
                    yw[4] = (double)Y[wrapN(i0 + j + 3, N) * kDensePitch + cown];
                }
                if (j < 2) edge[j] = r;
                else if (j >= KT - 2) edge[j - KT + 4] = r;
                else Y[(i0 + j) * kDensePitch + cown] = r;   // own rows, already in the window
            }
            __syncthreads();
            Y[i0 * kDensePitch + cown] = edge[0];
            Y[(i0 + 1) * kDensePitch + cown] = edge[1];
            Y[(i0 + KT - 2) * kDensePitch + cown] = edge[2];
            Y[(i0 + KT - 1) * kDensePitch + cown] = edge[3];
        }
        __syncthreads();

        // 4. y = yhat + R r (R = A^-1 in one BF16 term), accumulated onto yhat
#pragma unroll 1
        for (int k0 = 0; k0 < N; k0 += 32) {
            bf16x8 rb[2];
#pragma unroll
            for (int sub = 0; sub < 2; ++sub)
#pragma unroll
                for (int t = 0; t < 8; ++t) rb[sub][t] = (__bf16)Y[(k0 + 8 * q + t) * kDensePitch + 16 * sub + r16];
#pragma unroll
            for (int j = 0; j < SPW; ++j) {
                const int s = w + 4 * j;
                if (s < NSTRIP) {
                    const int start = kDenseExt + wrapN(k0 - 16 * s, N) + 8 * q - r16;
                    const bf16x8 a = circ_frag(rhi, start);
#pragma unroll
                    for (int sub = 0; sub < 2; ++sub)
                        acc[j][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, rb[sub], acc[j][sub], 0, 0, 0);
                }
            }
        }
        // 5. results through the tile to coalesced stores
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SPW; ++j) {
            const int s = w + 4 * j;
            if (s < NSTRIP)
#pragma unroll
                for (int sub = 0; sub < 2; ++sub)
#pragma unroll
                    for (int t = 0; t < 4; ++t) F[(16 * s + 4 * q + t) * kDensePitch + 16 * sub + r16] = acc[j][sub][t];
        }
        __syncthreads();
        {
            float *obase = out + pd.out_base[0] + (int64_t)wi.field * pd.out_fstride;
            const int64_t osd = pd.osd;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                int i, c;
                dense_elem<N, XDIR>(tid, k, i, c);
                const int64_t o = col_out[buf][c];
                if (o >= 0)
                    __builtin_nontemporal_store(F[i * kDensePitch + c],
                                                obase + o + (XDIR ? (int64_t)i : (int64_t)i * osd));
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_dense_form(int ntab, const void *tabs, const double *coefs, unsigned char *out, double *scratch,
                             int64_t scratch_per, int *status, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_form, dim3(ntab), dim3(256), 0, st, (const DenseTab *)tabs, coefs, 0.0, out, scratch,
                       scratch_per, status);
    return hipGetLastError();
}

template <int N, bool XDIR>
static const void *dense_fn() {
    return reinterpret_cast<const void *>(&k_dense_apply<N, XDIR>);
}

// Kernel of one (line length, x or not) class; nullptr for an unsupported N.
const void *dense_apply_fn(int N, bool xdir) {
    switch (N) {
#define CFD_DENSE_N(n) \
    case n: return xdir ? dense_fn<n, true>() : dense_fn<n, false>();
        CFD_DENSE_N(32) CFD_DENSE_N(64) CFD_DENSE_N(96) CFD_DENSE_N(128)
        CFD_DENSE_N(160) CFD_DENSE_N(192) CFD_DENSE_N(224) CFD_DENSE_N(256)
#undef CFD_DENSE_N
    default: return nullptr;
    }
}

hipError_t launch_dense_apply(const void *fn, int grid, hipStream_t st, const void *items, int nitems,
                              const PassDesc *passes, const void *tabs, const unsigned char *tabdata, const float *in,
                              float *out) {
    const DenseItem *it = (const DenseItem *)items;
    const DenseTab *tb = (const DenseTab *)tabs;
    void *args[] = {(void *)&it, (void *)&nitems, (void *)&passes, (void *)&tb, (void *)&tabdata, (void *)&in,
                    (void *)&out};
    return hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, st);
}

size_t dense_tab_bytes(int N) { return 16 * sizeof(double) + 3 * (size_t)(N + 48) * 2; }
size_t dense_tab_struct_size() { return sizeof(DenseTab); }
size_t dense_item_size() { return sizeof(DenseItem); }
void fill_dense_tab(void *dst, int N, int nl, int m, int64_t off) {
    DenseTab t;
    t.N = N; t.nl = nl; t.m = m; t.pad = 0; t.off = off;
    *reinterpret_cast<DenseTab *>(dst) = t;
}
void fill_dense_item(void *dst, int pass, int field, int line0, int tab) {
    DenseItem d{pass, field, line0, tab};
    *reinterpret_cast<DenseItem *>(dst) = d;
}

}  // namespace cfd
