// Dense mixed-precision operator for periodic lines (gfx950).
//
// On a periodic line the compact operator is the circulant matrix
// D = h^-d A^-1 B (the periodic D of Sec. 2.2, formed explicitly as the paper
// remarks one may do with the inverse matrix, Sec. 2.6).  This path:
//   * forms A^-1 B and A^-1 in FP64 on the GPU (dense Gauss-Jordan on
//     [A | B | I], k_dense_form) and keeps row 0 of each (a circulant matrix
//     is its first row): D[i][j] = m[(j - i) mod N], R[i][j] = rho[(j - i) mod N];
//   * splits m into BF16 hi + lo terms and rho into a BF16 hi term, and marks
//     the 16 x 32 circulant blocks whose entries are not negligible;
//   * per wave and 16 lines: yhat = D_hi f_hi + D_hi f_lo + D_lo f_hi over
//     those blocks on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation), then
//     one refinement with the FP64 banded residual r = h^-d B f - A yhat and
//     y = yhat + R_hi r accumulated into the same registers.
// Inputs and outputs are FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kDenseExt = 16;          // wrap-around margin of the extended circulant rows

// Layout of one dense table (per scheme and line length), in bytes:
//   double coefs[16]:  b_{-5..5} (interior stencil), alpha_{-2..2}
//   bf16 mhi[N+48], mlo[N+48], rhi[N+48]: extended circulant rows,
//       ext[kDenseExt + k] = row[k mod N] for k in [-16, N+32)
//   uint32 mask[3]: significant 16 x 32 circulant blocks of each term (bit w)
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
    // significant circulant blocks: the 16 x 32 block w of a term holds the row
    // entries at offsets 16 w - 15 .. 16 w + 31; it is kept if one of them
    // reaches 2^-24 of the row's largest entry (A^-1 B and A^-1 decay
    // geometrically away from the diagonal; the FP64 residual refinement
    // absorbs what the dropped blocks leave in yhat)
    if (threadIdx.x == 0) {
        double dmax = 0.0, rmax = 0.0;
        for (int k = 0; k < N; ++k) {
            dmax = fmax(dmax, fabs(M[k + N]));
            rmax = fmax(rmax, fabs(M[k + 2 * N]));
        }
        const double thr = dmax * 0x1p-24, thr_r = rmax * 0x1p-24;
        uint32_t mk[3] = {0u, 0u, 0u};
        for (int w = 0; w < N / 16; ++w)
            for (int o = -15; o <= 31; ++o) {
                const int k = wrapN(16 * w + o, N);
                const double d = M[k + N], r = M[k + 2 * N];
                const double lo = d - (double)(float)(__bf16)(float)d;
                if (fabs(d) >= thr) mk[0] |= 1u << w;
                if (fabs(lo) >= thr) mk[1] |= 1u << w;
                if (fabs(r) >= thr_r) mk[2] |= 1u << w;
            }
        uint32_t *mo = reinterpret_cast<uint32_t *>(base + 16 * sizeof(double) + 3 * (size_t)(N + 48) * 2);
        for (int k = 0; k < 3; ++k) mo[k] = mk[k];
        status[blockIdx.x] = bad;
    }
}

// ---------------------------------------------------------------------------
// Apply
//
// A workgroup takes an item of 64 lines; each of its four waves owns 16 of
// them (one MFMA column block) and works on its own, with no workgroup
// barrier except when the item's table differs from the one staged.  Two
// workgroups share a CU, so one wave's matrix-core work overlaps another's
// FP64 residual.  Per wave and item:
//   1. its lines' inputs, read in the B-operand layout (lane (q, c) holds
//      nodes 32 kb + 8 q + t of line c), go to its LDS tile F and are split
//      into BF16 hi / lo fragments;
//   2. yhat = D f: the 16 x 32 block of D at strip s, column block kb depends
//      only on w = (2 kb - s) mod N/16, so the loop runs over w with the two
//      A fragments of w (hi, lo) live and meets every kb once; blocks the
//      table marks as negligible are skipped;
//   3. FP64 residual r = h^-d B f - A yhat in the accumulator layout (lane
//      (q, c) holds rows 16 s + 4 q .. + 3 of line c): yhat's neighbour rows
//      come from the lanes 16 above and below, f from F; r goes to LDS as
//      BF16 over the part of F no later strip reads;
//   4. y = yhat + R r with R's fragments and the same loop;
//   5. stores straight from the accumulators.
// ---------------------------------------------------------------------------
struct DenseItem {
    int32_t pass;
    int32_t field;
    int32_t line0;
    int32_t tab;
};

constexpr int kDenseWaves = 4;
constexpr int kDenseLinesW = 16;                              // lines per wave
constexpr int kDenseItemLines = kDenseWaves * kDenseLinesW;   // lines per item

// LDS geometry of one line length.
//  * per-wave tile F: 16 lines x FP floats, FP = N + 4 (FP / 4 odd: the 16
//    lanes of a quarter-wave reading 16 B at one node of 16 lines hit
//    distinct banks);
//  * circulant tables: per term (D_hi, D_lo, R_hi) eight skewed copies
//    E_j[x] = row[(x - j - 16) mod N], x < 2 SPD, SPD dwords apart; lane
//    (q, c) reads its 8 entries of fragment w at E_{c % 8}[16 + 8 q - 8 (c / 8) + 16 w],
//    a 16-byte-aligned position.  SPD is an odd multiple of 8, which spreads
//    the 16 lanes of a quarter-wave over all banks.
template <int N>
struct DenseGeom {
    static constexpr int NW = N / 16;   // strips = distinct circulant blocks per term
    static constexpr int NK = N / 32;   // 32-wide column blocks
    static constexpr int FP = N + 4;
    static constexpr int SPD0 = ((N + 32) / 2 + 7) / 8 * 8;
    static constexpr int SPD = (SPD0 / 8) % 2 ? SPD0 : SPD0 + 8;
    static constexpr int TILE = kDenseLinesW * FP;                // floats per wave
    static constexpr int LDS = kDenseWaves * TILE + 3 * 8 * SPD;  // dwords
};

__device__ __forceinline__ bf16x8 split_hi(const float (&v)[8], bf16x8 &lo) {
    bf16x8 hi;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const __bf16 h = (__bf16)v[t];
        hi[t] = h;
        lo[t] = (__bf16)(v[t] - (float)h);
    }
    return hi;
}

// Two FP32 values to packed BF16 (round to nearest even), a in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const __bf16 x = (__bf16)a, y = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(unsigned short, x) | ((uint32_t)__builtin_bit_cast(unsigned short, y) << 16);
}

template <int N, bool XDIR, int MR>
__global__ void __launch_bounds__(64 * kDenseWaves) __attribute__((amdgpu_waves_per_eu(2)))
k_dense_apply(const DenseItem *__restrict__ items, int nitems, const PassDesc *__restrict__ passes,
              const DenseTab *__restrict__ tabs, const unsigned char *__restrict__ tabdata,
              const float *__restrict__ in, float *__restrict__ out) {
    using G = DenseGeom<N>;
    constexpr int NW = G::NW, NK = G::NK, FP = G::FP, SPD = G::SPD;
    __shared__ __attribute__((aligned(16))) float smem[G::LDS];
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63;
    const int q = l >> 4, c = l & 15;
    float *Fw = smem + w * G::TILE;
    unsigned short *Fb = reinterpret_cast<unsigned short *>(Fw);   // r as BF16 over F, pitch 2 FP
    unsigned short *T = reinterpret_cast<unsigned short *>(smem + kDenseWaves * G::TILE);
    const int fbase_lane = (c & 7) * 2 * SPD + 16 + 8 * q - 8 * (c >> 3);   // BF16 index, fragment 0
    const int addr_dn = ((l - 16) & 63) << 2;   // ds_bpermute address of lane l - 16
    const int addr_up = ((l + 16) & 63) << 2;   // of lane l + 16

    // this lane's line of an item (lines past the last one compute on line0 and
    // store nothing); byte offsets within the field stay below 2^32 (checked at
    // plan creation)
    auto line_of = [&](const DenseItem &wi, const PassDesc &pd, uint32_t &oi, uint32_t &oo) {
        int line = wi.line0 + w * kDenseLinesW + c;
        const bool live = line < pd.nlines;
        if (!live) line = wi.line0;
        const int lu = line % pd.nu, lv = line / pd.nu;
        oi = 4u * (uint32_t)(lv * pd.sv + lu * pd.su);
        oo = 4u * (uint32_t)(lv * pd.osv + lu * pd.osu);
        return live;
    };
    // an item's inputs: node 32 kb + 8 q + t of line c
    float pre[NK][8];
    auto load_item = [&](const DenseItem &wi) {
        const PassDesc &pd = passes[wi.pass];
        uint32_t oi, oo;
        (void)line_of(wi, pd, oi, oo);
        const char *fb = reinterpret_cast<const char *>(in + pd.in_base + (int64_t)(pd.field0 + wi.field) * pd.in_fstride);
        if constexpr (XDIR) {
            const bool al = ((reinterpret_cast<uintptr_t>(fb) & 15) == 0) && ((pd.su & 3) == 0) && ((pd.sv & 3) == 0);
            const uint32_t o0 = oi + 32u * q;
            if (al) {
#pragma unroll
                for (int kb = 0; kb < NK; ++kb)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float4 v = *reinterpret_cast<const float4 *>(fb + o0 + 128u * kb + 16u * h);
                        pre[kb][4 * h] = v.x;
                        pre[kb][4 * h + 1] = v.y;
                        pre[kb][4 * h + 2] = v.z;
                        pre[kb][4 * h + 3] = v.w;
                    }
            } else {
#pragma unroll
                for (int kb = 0; kb < NK; ++kb)
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        pre[kb][t] = *reinterpret_cast<const float *>(fb + o0 + 128u * kb + 4u * t);
            }
        } else {
            const uint32_t sdb = 4u * (uint32_t)pd.sd;
            const uint32_t o0 = oi + 8u * q * sdb;
#pragma unroll
            for (int kb = 0; kb < NK; ++kb)
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    pre[kb][t] = *reinterpret_cast<const float *>(fb + o0 + (uint32_t)(32 * kb + t) * sdb);
        }
    };

    int cur_tab = -1;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const DenseItem wi = items[it];
        const PassDesc &pd = passes[wi.pass];
        const DenseTab tb = tabs[wi.tab];
        // circulant tables of this item's scheme (all waves hold the same item)
        if (wi.tab != cur_tab) {
            __syncthreads();   // every wave is done with the previous table
            const unsigned short *rows = reinterpret_cast<const unsigned short *>(tabdata + tb.off + 16 * sizeof(double));
            for (int e = tid; e < 3 * 8 * 2 * SPD; e += 64 * kDenseWaves) {
                const int term = e / (16 * SPD);
                const int rem = e - term * 16 * SPD;
                const int j = rem / (2 * SPD);
                const int x = rem - j * 2 * SPD;
                int k = (x - j - 16) % N;
                if (k < 0) k += N;
                T[e] = rows[term * (N + 48) + kDenseExt + k];
            }
            __syncthreads();
            cur_tab = wi.tab;
        }
        uint32_t oi, oo;
        const bool live = line_of(wi, pd, oi, oo);

        // 1. inputs (the other workgroup on the CU covers their latency; a
        //    prefetch one item ahead measured slower)
        load_item(wi);
        // to F (B layout, 16 B per write) and BF16 hi / lo fragments
#pragma unroll
        for (int kb = 0; kb < NK; ++kb)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                *reinterpret_cast<float4 *>(Fw + c * FP + 32 * kb + 8 * q + 4 * h) =
                    make_float4(pre[kb][4 * h], pre[kb][4 * h + 1], pre[kb][4 * h + 2], pre[kb][4 * h + 3]);
        bf16x8 bh[NK], bl[NK];
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) bh[kb] = split_hi(pre[kb], bl[kb]);

        // 2. yhat = D_hi f_hi + D_hi f_lo + D_lo f_hi over the significant blocks
        const uint32_t *mask = reinterpret_cast<const uint32_t *>(tabdata + tb.off + 16 * sizeof(double) +
                                                                  3 * (size_t)(N + 48) * 2);
        const uint32_t m_hi = mask[0], m_lo = mask[1], m_r = mask[2];
        f32x4 acc[NW];
#pragma unroll
        for (int s = 0; s < NW; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int wb = 0; wb < NW; ++wb) {
            if (m_hi & (1u << wb)) {
                const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(T + fbase_lane + 16 * wb);
#pragma unroll
                for (int kb = 0; kb < NK; ++kb) {
                    const int s = (2 * kb - wb + NW) % NW;
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[kb], acc[s], 0, 0, 0);
                }
#pragma unroll
                for (int kb = 0; kb < NK; ++kb) {
                    const int s = (2 * kb - wb + NW) % NW;
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[kb], acc[s], 0, 0, 0);
                }
            }
            if (m_lo & (1u << wb)) {
                const bf16x8 al = *reinterpret_cast<const bf16x8 *>(T + 16 * SPD + fbase_lane + 16 * wb);
#pragma unroll
                for (int kb = 0; kb < NK; ++kb) {
                    const int s = (2 * kb - wb + NW) % NW;
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[kb], acc[s], 0, 0, 0);
                }
            }
        }
        // 3. yhat = h^-d A^-1 B f; FP64 residual on rows 16 s + 4 q + t of line c
        const double hinv = pd.hinv[0];
        const float scale = (float)hinv;
#pragma unroll
        for (int s = 0; s < NW; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[s][t] *= scale;
        // the strip loop for RHS half-width up to MR (3 covers the interior
        // schemes of Sec. 2 with fewer FMAs and LDS reads; 5 any stencil the
        // tables hold)
        {
            constexpr int NCH = MR <= 3 ? 3 : 5;   // 4-row chunks of f per strip
            constexpr int C0 = 4 * (NCH / 2);      // rows of f before the strip's first row
            const double *cf = reinterpret_cast<const double *>(tabdata + tb.off);
            double cb[2 * MR + 1], ca[5];
#pragma unroll
            for (int t = 0; t < 2 * MR + 1; ++t) cb[t] = cf[5 - MR + t] * hinv;
#pragma unroll
            for (int t = 0; t < 5; ++t) ca[t] = cf[11 + t];
            const f32x4 *Fl4 = reinterpret_cast<const f32x4 *>(Fw + c * FP);   // 16-byte reads (FP % 4 == 0)
            uint32_t r01[2][2];   // strips 0 and 1: F rows they would overwrite are read by the last strip
#pragma unroll
            for (int s = 0; s < NW; ++s) {
                const int sm = (s + NW - 1) % NW, sp = (s + 1) % NW;
                // yhat rows 16 s + 4 q - 2 .. + 5: two from lane l - 16 (q = 0: strip s - 1
                // of lane q = 3), four own, two from lane l + 16 (q = 3: strip s + 1 of q = 0)
                const float dn2 = q == 3 ? acc[sm][2] : acc[s][2];
                const float dn3 = q == 3 ? acc[sm][3] : acc[s][3];
                const float up0 = q == 0 ? acc[sp][0] : acc[s][0];
                const float up1 = q == 0 ? acc[sp][1] : acc[s][1];
                double yw[8];
                yw[0] = (double)__builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr_dn, __builtin_bit_cast(int, dn2)));
                yw[1] = (double)__builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr_dn, __builtin_bit_cast(int, dn3)));
#pragma unroll
                for (int t = 0; t < 4; ++t) yw[2 + t] = (double)acc[s][t];
                yw[6] = (double)__builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr_up, __builtin_bit_cast(int, up0)));
                yw[7] = (double)__builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr_up, __builtin_bit_cast(int, up1)));
                // f rows 16 s + 4 q - C0 .. 16 s + 4 q - C0 + 4 NCH - 1
                float fw[4 * NCH];
#pragma unroll
                for (int k = 0; k < NCH; ++k) {
                    f32x4 v = Fl4[((16 * s + 4 * q - C0 + 4 * k + N) % N) >> 2];
                    if (k == 0 || k == NCH - 1) __asm__ volatile("" : "+v"(v));   // one 16-byte read, not a narrowed one
#pragma unroll
                    for (int e = 0; e < 4; ++e) fw[4 * k + e] = v[e];
                }
                float rr[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    double bf = 0.0, ay = 0.0;
#pragma unroll
                    for (int m = 0; m < 2 * MR + 1; ++m) bf = fma(cb[m], (double)fw[C0 - MR + t + m], bf);
#pragma unroll
                    for (int m = 0; m < 5; ++m) ay = fma(ca[m], yw[t + m], ay);
                    float rf = (float)(bf - ay);
                    __asm__ volatile("" : "+v"(rf));   // keeps the f64 -> f32 -> bf16 rounding in two plain steps
                    rr[t] = rf;
                }
                const uint32_t p0 = pack_bf16(rr[0], rr[1]), p1 = pack_bf16(rr[2], rr[3]);
                if (s < 2) {
                    r01[s][0] = p0;
                    r01[s][1] = p1;
                } else {
                    // BF16 rows 16 s + 4 q .. + 3 of line c sit over F rows 8 s + 2 q .. + 1,
                    // which no later strip reads
                    *reinterpret_cast<uint2 *>(Fb + c * 2 * FP + 16 * s + 4 * q) = make_uint2(p0, p1);
                }
            }
#pragma unroll
            for (int s = 0; s < 2 && s < NW; ++s)
                *reinterpret_cast<uint2 *>(Fb + c * 2 * FP + 16 * s + 4 * q) = make_uint2(r01[s][0], r01[s][1]);
        }
        __builtin_amdgcn_wave_barrier();
        bf16x8 rb[NK];
#pragma unroll
        for (int kb = 0; kb < NK; ++kb) rb[kb] = *reinterpret_cast<const bf16x8 *>(Fb + c * 2 * FP + 32 * kb + 8 * q);

        // 4. y = yhat + R r (R = A^-1 in one BF16 term)
#pragma unroll
        for (int wb = 0; wb < NW; ++wb) {
            if (m_r & (1u << wb)) {
                const bf16x8 ar = *reinterpret_cast<const bf16x8 *>(T + 32 * SPD + fbase_lane + 16 * wb);
#pragma unroll
                for (int kb = 0; kb < NK; ++kb) {
                    const int s = (2 * kb - wb + NW) % NW;
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, rb[kb], acc[s], 0, 0, 0);
                }
            }
        }
        // 5. stores: rows 16 s + 4 q .. + 3 of line c
        if (live) {
            char *ob = reinterpret_cast<char *>(out + pd.out_base[0] + (int64_t)wi.field * pd.out_fstride);
            if constexpr (XDIR) {
                char *dst = ob + oo + 16u * q;
                if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
#pragma unroll
                    for (int s = 0; s < NW; ++s)
                        __builtin_nontemporal_store(acc[s], reinterpret_cast<f32x4 *>(dst + 64 * s));
                } else {
#pragma unroll
                    for (int s = 0; s < NW; ++s)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            __builtin_nontemporal_store(acc[s][t], reinterpret_cast<float *>(dst + 64 * s + 4 * t));
                }
            } else {
                const uint32_t osdb = 4u * (uint32_t)pd.osd;
                const uint32_t o0 = oo + 4u * q * osdb;
#pragma unroll
                for (int s = 0; s < NW; ++s)
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        __builtin_nontemporal_store(acc[s][t],
                                                    reinterpret_cast<float *>(ob + o0 + (uint32_t)(16 * s + t) * osdb));
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_dense_form(int ntab, const void *tabs, const double *coefs, unsigned char *out, double *scratch,
                             int64_t scratch_per, int *status, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_form, dim3(ntab), dim3(256), 0, st, (const DenseTab *)tabs, coefs, 0.0, out, scratch,
                       scratch_per, status);
    return hipGetLastError();
}

template <int N, bool XDIR, int MR>
static const void *dense_fn() {
    return reinterpret_cast<const void *>(&k_dense_apply<N, XDIR, MR>);
}

template <int N>
static const void *dense_fn(bool xdir, bool wide) {
    if (wide) return xdir ? dense_fn<N, true, 5>() : dense_fn<N, false, 5>();
    return xdir ? dense_fn<N, true, 3>() : dense_fn<N, false, 3>();
}

// Kernel of one (line length, x or not, RHS half-width above 3 or not) class;
// nullptr for an unsupported N.
const void *dense_apply_fn(int N, bool xdir, bool wide) {
    switch (N) {
#define CFD_DENSE_N(n) \
    case n: return dense_fn<n>(xdir, wide);
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

size_t dense_tab_bytes(int N) { return 16 * sizeof(double) + 3 * (size_t)(N + 48) * 2 + 4 * sizeof(uint32_t); }
size_t dense_tab_struct_size() { return sizeof(DenseTab); }
size_t dense_item_size() { return sizeof(DenseItem); }
int dense_item_lines() { return kDenseItemLines; }
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
