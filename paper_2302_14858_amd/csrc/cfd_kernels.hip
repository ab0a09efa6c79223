// Device kernels of the MI355X compact finite-difference library (gfx950).
//
// Line operator (arXiv 2302.14858, Eq. sch_cent_om and its matrix form
// Eqs. diff_mat_subL / diff_mat_subR): on every grid line of N nodes the
// derivative f~ solves  D_L f~ = h^-d D_R f,  where D_L has identity rows on
// the block-closure rows and the banded alpha^(d) rows elsewhere, and D_R has
// the explicit closure stencil or the interior stencil alpha^(0).  Periodic
// lines use the circulant operator instead.
//
// GPU decomposition (not from the paper, whose TDMA runs one line at a time):
//  * a line is cut into P partitions of L = N/P consecutive rows;
//  * one wavefront owns one partition of 64 lines: lane = line, so loads and
//    stores along y and z are coalesced across the wavefront and every table
//    entry a wavefront reads is uniform (scalar loads);
//  * each lane streams its partition once: the RHS stencil is evaluated from a
//    register ring and fused with forward elimination, then back substitution
//    gives the partition-local solution y;
//  * the partitions are coupled through 2*nl boundary unknowns each.  Their
//    values follow from the boundary entries of every partition's y by one
//    fixed linear map (rows of the inverse reduced system); the lanes of a
//    line exchange those entries through LDS and correct
//    x = y - sum(boundary value * spike vector).  For periodic lines the same
//    algebra closes the wrap-around, which is the Woodbury form of the cyclic
//    solve.
// All line-independent quantities (local LU factors, spikes, reduced-system
// rows) are built once per plan in FP64 by k_build_tables.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

// ---------------------------------------------------------------------------
// Line kernel
// ---------------------------------------------------------------------------
//   T     storage and arithmetic type
//   NL    implicit half-width (0 explicit, 1 tri, 2 penta)
//   L     rows per partition
//   NOPS  operators sharing one pass over the input (same field, direction)
//   PAR   bit o set: operator o has an antisymmetric interior stencil (odd d)
//   MI    interior stencil half-width
//   HW    ring half-width = max(MI, closure half-width)
template <typename T, int NL, int L, int NOPS, int PAR, int MI, int HW>
__global__ void __launch_bounds__(512)
k_lines(const WorkItem *__restrict__ items, int nitems, const PassDesc *__restrict__ passes,
        const T *__restrict__ tabs, const int64_t *__restrict__ taboff, const T *__restrict__ in,
        T *__restrict__ out)
{
    static_assert(NL == 0 || L >= 2 * NL, "partition too short");
    constexpr int R = 2 * HW + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);

    const int P = blockDim.x >> 6;
    const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = threadIdx.x & 63;
    const int B = 2 * NL * P;
    const int Bp = B | 1;

    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const WorkItem wi = items[it];
        const PassDesc &pd = passes[wi.pass];
        const int N = pd.N;
        const int ng = pd.ng;
        const bool periodic = pd.periodic != 0;

        int line = wi.line0 + g;
        const bool active = line < pd.nlines;
        if (!active) line = pd.nlines - 1;
        const int lu = line % pd.nu;
        const int lv = line / pd.nu;
        const T *src = in + pd.in_base + (int64_t)(pd.field0 + wi.field) * pd.in_fstride +
                       (int64_t)lv * pd.sv + (int64_t)lu * pd.su;
        const int64_t sd = pd.sd;
        const int k0 = p * L;

        const T *tb[NOPS];
#pragma unroll
        for (int o = 0; o < NOPS; ++o) tb[o] = tabs + taboff[pd.tab[o]];

        // node j of this line; out-of-block nodes read as 0 (their weights are 0)
        auto load = [&](int j) -> T {
            if (periodic) {
                if (j < 0) j += N;
                if (j >= N) j -= N;
                return src[(int64_t)j * sd];
            }
            if (j < -ng || j >= N + ng) return T(0);
            return src[(int64_t)j * sd];
        };

        T f[R];
#pragma unroll
        for (int t = 0; t < R - 1; ++t) f[t] = load(k0 - HW + t);

        T y[NOPS][L];
        const bool first = (p == 0) && !periodic;
        const bool last = (p == P - 1) && !periodic;

#pragma unroll
        for (int i = 0; i < L; ++i) {
            f[R - 1] = load(k0 + i + HW);
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                const T *cf = tb[o];
                T r;
                if ((PAR >> o) & 1) {  // constant after unrolling
                    r = T(0);
#pragma unroll
                    for (int m = 1; m <= MI; ++m) r += cf[kCoefA + 5 + m] * (f[HW + m] - f[HW - m]);
                } else {
                    r = cf[kCoefA + 5] * f[HW];
#pragma unroll
                    for (int m = 1; m <= MI; ++m) r += cf[kCoefA + 5 + m] * (f[HW + m] + f[HW - m]);
                }
                if constexpr (NL > 0) {
                    // explicit closure rows (identity rows of D_L)
                    if (i < NL && first) {
                        const T *c = cf + kCoefCL + i * 11;
                        T s = T(0);
#pragma unroll
                        for (int m = -HW; m <= HW; ++m) s += c[5 + m] * f[HW + m];
                        r = s;
                    }
                    if (i >= L - NL && last) {
                        const T *c = cf + kCoefCR + (L - 1 - i) * 11;
                        T s = T(0);
#pragma unroll
                        for (int m = -HW; m <= HW; ++m) s += c[5 + m] * f[HW + m];
                        r = s;
                    }
                    // forward elimination with the partition-local factors
                    const T *fac = cf + kCoefHdr + (int64_t)(k0 + i) * 5;
                    if (i >= 1) r -= fac[0] * y[o][i - 1];
                    if (NL >= 2 && i >= 2) r -= fac[1] * y[o][i - 2];
                }
                y[o][i] = r;
            }
#pragma unroll
            for (int t = 0; t < R - 1; ++t) f[t] = f[t + 1];
        }

        if constexpr (NL > 0) {
            // back substitution
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                const T *cf = tb[o];
#pragma unroll
                for (int i = L - 1; i >= 0; --i) {
                    const T *fac = cf + kCoefHdr + (int64_t)(k0 + i) * 5;
                    T v = y[o][i];
                    if (i + 1 < L) v -= fac[2] * y[o][i + 1];
                    if (NL >= 2 && i + 2 < L) v -= fac[3] * y[o][i + 2];
                    y[o][i] = v * fac[4];
                }
            }
            // coupling of the partitions (and the periodic wrap)
            if (periodic || P > 1) {
                // boundary slots: rows 0..NL-1 and L-NL..L-1 of every partition
#pragma unroll
                for (int o = 0; o < NOPS; ++o) {
                    T *row = lds + ((int64_t)o * 64 + g) * Bp + p * 2 * NL;
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        row[t] = y[o][t];
                        row[NL + t] = y[o][L - NL + t];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int o = 0; o < NOPS; ++o) {
                    const T *cf = tb[o];
                    const int Lrows = N;  // fac occupies N*5 entries
                    const T *spk = cf + kCoefHdr + (int64_t)Lrows * 5 + (int64_t)p * 2 * NL * L;
                    const T *krow = cf + kCoefHdr + (int64_t)Lrows * 5 + (int64_t)P * 2 * NL * L +
                                    (int64_t)p * 2 * NL * B;
                    const T *row = lds + ((int64_t)o * 64 + g) * Bp;
                    T xq[2 * NL];
#pragma unroll
                    for (int q = 0; q < 2 * NL; ++q) xq[q] = T(0);
                    for (int b = 0; b < B; ++b) {
                        const T yb = row[b];
#pragma unroll
                        for (int q = 0; q < 2 * NL; ++q) xq[q] += krow[q * B + b] * yb;
                    }
#pragma unroll
                    for (int i = 0; i < L; ++i) {
                        T v = y[o][i];
#pragma unroll
                        for (int q = 0; q < 2 * NL; ++q) v -= xq[q] * spk[q * L + i];
                        y[o][i] = v;
                    }
                }
                __syncthreads();  // LDS is reused by the next item
            }
        }

        if (active) {
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                T *dst = out + pd.out_base[o] + (int64_t)wi.field * pd.out_fstride + (int64_t)lv * pd.osv +
                         (int64_t)lu * pd.osu;
                const T hinv = (T)pd.hinv[o];
#pragma unroll
                for (int i = 0; i < L; ++i) dst[(int64_t)(k0 + i) * pd.osd] = y[o][i] * hinv;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Table construction, FP64, one thread per table
// ---------------------------------------------------------------------------
struct TabSpec {
    int N, P, L, nl, nc, periodic;
    double alpha[2 * kMaxNL + 1];
    int64_t off;   // element offset of the table (coefficient block first)
};

// Entry of D_L in global row k at unwrapped offset o (column k + o).
__device__ inline double dl_entry(const TabSpec &s, int k, int o) {
    const bool ident = !s.periodic && (k < s.nc || k >= s.N - s.nc);
    if (ident) return o == 0 ? 1.0 : 0.0;
    if (o < -s.nl || o > s.nl) return 0.0;
    if (!s.periodic && (k + o < 0 || k + o >= s.N)) return 0.0;
    return s.alpha[kMaxNL + o];
}

// Solve with partition-local factors (in place), the same recurrences the
// line kernel runs.
__device__ inline void local_solve(const double *fac, int L, int nl, double *v) {
    for (int i = 0; i < L; ++i) {
        double r = v[i];
        if (i >= 1) r -= fac[i * 5 + 0] * v[i - 1];
        if (nl >= 2 && i >= 2) r -= fac[i * 5 + 1] * v[i - 2];
        v[i] = r;
    }
    for (int i = L - 1; i >= 0; --i) {
        double r = v[i];
        if (i + 1 < L) r -= fac[i * 5 + 2] * v[i + 1];
        if (nl >= 2 && i + 2 < L) r -= fac[i * 5 + 3] * v[i + 2];
        v[i] = r * fac[i * 5 + 4];
    }
}

__global__ void k_build_tables(int ntab, const TabSpec *__restrict__ specs, double *__restrict__ data,
                               double *__restrict__ scratch, int64_t scratch_per, int *__restrict__ status)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab) return;
    const TabSpec s = specs[t];
    double *tab = data + s.off;
    double *fac = tab + kCoefHdr;
    const int N = s.N, P = s.P, L = s.L, nl = s.nl;
    if (nl == 0) { status[t] = 0; return; }
    const int B = 2 * nl * P;
    double *spk = fac + (int64_t)N * 5;
    double *krow = spk + (int64_t)P * 2 * nl * L;
    double *K = scratch + (int64_t)t * scratch_per;      // B x B
    double *Kinv = K + (int64_t)B * B;                   // B x B
    double *v = Kinv + (int64_t)B * B;                   // L
    int bad = 0;

    // 1. partition-local banded LU without pivoting (Doolittle, nl <= 2)
    for (int p = 0; p < P; ++p) {
        double *F = fac + (int64_t)p * L * 5;
        for (int i = 0; i < L; ++i) {
            const int k = p * L + i;
            auto a = [&](int o) -> double {   // local entry (row i, col i+o), in partition only
                if (i + o < 0 || i + o >= L) return 0.0;
                return dl_entry(s, k, o);
            };
            double l2 = 0, l1 = 0;
            if (nl >= 2 && i >= 2) l2 = a(-2) / (1.0 / F[(i - 2) * 5 + 4]);
            if (i >= 1) {
                double num = a(-1);
                if (nl >= 2 && i >= 2) num -= l2 * F[(i - 2) * 5 + 2];
                l1 = num / (1.0 / F[(i - 1) * 5 + 4]);
            }
            double dd = a(0);
            if (i >= 1) dd -= l1 * F[(i - 1) * 5 + 2];
            if (nl >= 2 && i >= 2) dd -= l2 * F[(i - 2) * 5 + 3];
            double u1 = a(1);
            if (nl >= 2 && i >= 1) u1 -= l1 * F[(i - 1) * 5 + 3];
            double u2 = (nl >= 2) ? a(2) : 0.0;
            if (!(fabs(dd) > 1e-12)) bad = 1;
            F[i * 5 + 0] = l1;
            F[i * 5 + 1] = l2;
            F[i * 5 + 2] = u1;
            F[i * 5 + 3] = u2;
            F[i * 5 + 4] = 1.0 / dd;
        }
    }
    // 2. spike vectors: response of partition p to its nl left and nl right
    //    neighbour unknowns (columns pL - j and (p+1)L + j - 1, j = 1..nl)
    for (int p = 0; p < P; ++p) {
        for (int q = 0; q < 2 * nl; ++q) {
            const bool left = q < nl;
            const int j = left ? q + 1 : q - nl + 1;
            for (int i = 0; i < L; ++i) {
                const int k = p * L + i;
                // unwrapped offset from row k to the neighbour column
                const int col = left ? p * L - j : (p + 1) * L + j - 1;
                const int o = col - k;
                double e = 0.0;
                if (o >= -nl && o <= nl) {
                    if (s.periodic || (col >= 0 && col < N)) e = dl_entry(s, k, o);
                    if (!s.periodic && (col < 0 || col >= N)) e = 0.0;
                }
                v[i] = e;
            }
            local_solve(fac + (int64_t)p * L * 5, L, nl, v);
            for (int i = 0; i < L; ++i) spk[((int64_t)p * 2 * nl + q) * L + i] = v[i];
        }
    }
    // 3. reduced system on the boundary slots: slot (p, t), t < nl -> row t,
    //    t >= nl -> row L - 2 nl + t.  (I + C) xb = yb.
    for (int i = 0; i < B * B; ++i) K[i] = 0.0;
    for (int i = 0; i < B; ++i) K[i * B + i] = 1.0;
    for (int p = 0; p < P; ++p) {
        const bool has_l = s.periodic || p > 0;
        const bool has_r = s.periodic || p < P - 1;
        const int pl = (p + P - 1) % P, pr = (p + 1) % P;
        for (int t = 0; t < 2 * nl; ++t) {
            const int rt = t < nl ? t : L - 2 * nl + t;
            const int row = p * 2 * nl + t;
            for (int j = 1; j <= nl; ++j) {
                if (has_l) K[row * B + pl * 2 * nl + (2 * nl - j)] += spk[((int64_t)p * 2 * nl + (j - 1)) * L + rt];
                if (has_r) K[row * B + pr * 2 * nl + (j - 1)] += spk[((int64_t)p * 2 * nl + nl + (j - 1)) * L + rt];
            }
        }
    }
    // Gauss-Jordan inverse with partial pivoting
    for (int i = 0; i < B * B; ++i) Kinv[i] = 0.0;
    for (int i = 0; i < B; ++i) Kinv[i * B + i] = 1.0;
    for (int c = 0; c < B; ++c) {
        int pv = c;
        for (int r = c + 1; r < B; ++r)
            if (fabs(K[r * B + c]) > fabs(K[pv * B + c])) pv = r;
        if (!(fabs(K[pv * B + c]) > 1e-14)) { bad = 1; break; }
        if (pv != c)
            for (int k = 0; k < B; ++k) {
                double x = K[c * B + k]; K[c * B + k] = K[pv * B + k]; K[pv * B + k] = x;
                x = Kinv[c * B + k]; Kinv[c * B + k] = Kinv[pv * B + k]; Kinv[pv * B + k] = x;
            }
        const double ip = 1.0 / K[c * B + c];
        for (int k = 0; k < B; ++k) { K[c * B + k] *= ip; Kinv[c * B + k] *= ip; }
        for (int r = 0; r < B; ++r) {
            if (r == c) continue;
            const double fct = K[r * B + c];
            if (fct == 0.0) continue;
            for (int k = 0; k < B; ++k) { K[r * B + k] -= fct * K[c * B + k]; Kinv[r * B + k] -= fct * Kinv[c * B + k]; }
        }
    }
    // 4. rows of K^-1 each partition needs: its nl left and nl right neighbour values
    for (int p = 0; p < P; ++p) {
        const bool has_l = s.periodic || p > 0;
        const bool has_r = s.periodic || p < P - 1;
        const int pl = (p + P - 1) % P, pr = (p + 1) % P;
        for (int q = 0; q < 2 * nl; ++q) {
            int src = -1;
            if (q < nl) { if (has_l) src = pl * 2 * nl + (2 * nl - (q + 1)); }
            else { if (has_r) src = pr * 2 * nl + (q - nl); }
            for (int b = 0; b < B; ++b)
                krow[((int64_t)p * 2 * nl + q) * B + b] = (src >= 0) ? Kinv[src * B + b] : 0.0;
        }
    }
    status[t] = bad;
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// Registry of compiled line-kernel variants
// ---------------------------------------------------------------------------
struct LineLaunch {
    int f32, nl, L, nops, par, mi, hw;
    const void *fn;
};

#define CFD_LK(T, F32, NL, L, NOPS, PAR, MI, HW) \
    {F32, NL, L, NOPS, PAR, MI, HW, reinterpret_cast<const void *>(&k_lines<T, NL, L, NOPS, PAR, MI, HW>)}

#define CFD_LK_BOTH(NL, L, NOPS, PAR, MI, HW) \
    CFD_LK(double, 0, NL, L, NOPS, PAR, MI, HW), CFD_LK(float, 1, NL, L, NOPS, PAR, MI, HW)

static const LineLaunch kLineKernels[] = {
    // pentadiagonal, first + second derivative fused (M = 3, closures of half-width 5)
    CFD_LK_BOTH(2, 8, 2, 1, 3, 5), CFD_LK_BOTH(2, 12, 2, 1, 3, 5), CFD_LK_BOTH(2, 16, 2, 1, 3, 5),
    CFD_LK_BOTH(2, 24, 2, 1, 3, 5),
    // tridiagonal, first + second derivative fused (M = 3, closures of half-width 4)
    CFD_LK_BOTH(1, 8, 2, 1, 3, 4), CFD_LK_BOTH(1, 16, 2, 1, 3, 4), CFD_LK_BOTH(1, 24, 2, 1, 3, 4),
    CFD_LK_BOTH(1, 32, 2, 1, 3, 4),
    // tridiagonal, one first derivative (M = 3 / M = 2)
    CFD_LK_BOTH(1, 8, 1, 1, 3, 4), CFD_LK_BOTH(1, 16, 1, 1, 3, 4), CFD_LK_BOTH(1, 24, 1, 1, 3, 4),
    CFD_LK_BOTH(1, 32, 1, 1, 3, 4),
    CFD_LK_BOTH(1, 8, 1, 1, 2, 4), CFD_LK_BOTH(1, 16, 1, 1, 2, 4), CFD_LK_BOTH(1, 32, 1, 1, 2, 4),
    // generic single-operator variants (any stencil up to half-width 5)
    CFD_LK_BOTH(1, 8, 1, 1, 5, 5), CFD_LK_BOTH(1, 16, 1, 1, 5, 5), CFD_LK_BOTH(1, 8, 1, 0, 5, 5),
    CFD_LK_BOTH(1, 16, 1, 0, 5, 5), CFD_LK_BOTH(2, 8, 1, 1, 5, 5), CFD_LK_BOTH(2, 16, 1, 1, 5, 5),
    CFD_LK_BOTH(2, 8, 1, 0, 5, 5), CFD_LK_BOTH(2, 16, 1, 0, 5, 5),
    // explicit schemes
    CFD_LK_BOTH(0, 8, 1, 1, 5, 5), CFD_LK_BOTH(0, 8, 1, 0, 5, 5),
};

const void *find_line_kernel(int f32, int nl, int L, int nops, int par, int mi, int hw, int *mi_out, int *hw_out) {
    // exact stencil match first, then the smallest generic variant that covers it
    const LineLaunch *best = nullptr;
    for (const LineLaunch &k : kLineKernels) {
        if (k.f32 != f32 || k.nl != nl || k.L != L || k.nops != nops || k.par != par) continue;
        if (k.mi < mi || k.hw < hw) continue;
        if (!best || (k.mi + k.hw) < (best->mi + best->hw)) best = &k;
    }
    if (!best) return nullptr;
    *mi_out = best->mi;
    *hw_out = best->hw;
    return best->fn;
}

// L values that have at least one compiled variant for (f32, nl, nops, par)
int line_kernel_Ls(int f32, int nl, int nops, int par, int mi, int hw, int *Ls, int cap) {
    int n = 0;
    for (const LineLaunch &k : kLineKernels) {
        if (k.f32 != f32 || k.nl != nl || k.nops != nops || k.par != par || k.mi < mi || k.hw < hw) continue;
        bool seen = false;
        for (int i = 0; i < n; ++i) seen |= (Ls[i] == k.L);
        if (!seen && n < cap) Ls[n++] = k.L;
    }
    return n;
}

hipError_t launch_lines(const void *fn, int grid, int P, size_t lds, hipStream_t st, const WorkItem *items,
                        int nitems, const PassDesc *passes, const void *tabs, const int64_t *taboff,
                        const void *in, void *out) {
    void *args[] = {(void *)&items, (void *)&nitems, (void *)&passes, (void *)&tabs,
                    (void *)&taboff, (void *)&in, (void *)&out};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * P), args, lds, st);
}

hipError_t launch_build_tables(int ntab, const void *specs, double *data, double *scratch, int64_t scratch_per,
                               int *status, hipStream_t st) {
    const TabSpec *sp = reinterpret_cast<const TabSpec *>(specs);
    hipLaunchKernelGGL(k_build_tables, dim3((ntab + 63) / 64), dim3(64), 0, st, ntab, sp, data, scratch,
                       scratch_per, status);
    return hipGetLastError();
}

hipError_t launch_to_f32(int64_t n, const double *a, float *b, hipStream_t st) {
    int grid = (int)((n + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(256), 0, st, n, a, b);
    return hipGetLastError();
}

size_t tabspec_size() { return sizeof(TabSpec); }

void fill_tabspec(void *dst, int N, int P, int L, int nl, int nc, int periodic, const double *alpha5, int64_t off) {
    TabSpec s;
    s.N = N; s.P = P; s.L = L; s.nl = nl; s.nc = nc; s.periodic = periodic;
    for (int i = 0; i < 2 * kMaxNL + 1; ++i) s.alpha[i] = alpha5[i];
    s.off = off;
    *reinterpret_cast<TabSpec *>(dst) = s;
}

}  // namespace cfd
