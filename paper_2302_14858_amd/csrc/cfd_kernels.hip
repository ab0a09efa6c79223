// Device kernels of the MI355X compact finite-difference library (gfx950):
// FP64 table construction, the registry of compiled line-kernel classes and
// the FP64 instantiations of the line kernel (cfd_lines.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "cfd_internal.h"
#include "cfd_kernels_reg.h"
#include "cfd_lines.h"

namespace cfd {

// ---------------------------------------------------------------------------
// Table construction, FP64, one thread per table
// ---------------------------------------------------------------------------
struct TabSpec {
    int N, P, L, nl, nc, periodic;   // line length, partitions, rows per partition (P L >= N)
    double alpha[2 * kMaxNL + 1];
    int64_t off;   // element offset of the table (coefficient block first)
    int ext;                         // implicit closure rows (iterated closure, nc = 1)
    double cl_d0, cl_up, gamma;      // their D_L entries and end-value weight
};

// Entry of D_L in global row k at unwrapped offset o (column k + o).  Rows
// past the line end (padding of the last partition) are identity rows, and
// so are the closure rows unless they are the implicit rows of an iterated
// closure: (cl_d0, cl_up) on row 0, mirrored on row N - 1.
__device__ inline double dl_entry(const TabSpec &s, int k, int o) {
    if (!s.periodic && k >= s.N) return o == 0 ? 1.0 : 0.0;
    const bool clo = !s.periodic && (k < s.nc || k >= s.N - s.nc);
    if (clo && s.ext) {
        if (o == 0) return s.cl_d0;
        return (k < s.nc ? o == 1 : o == -1) ? s.cl_up : 0.0;
    }
    if (clo) return o == 0 ? 1.0 : 0.0;
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
    const int N = s.N, P = s.P, L = s.L, nl = s.nl;
    if (nl == 0) { status[t] = 0; return; }
    const int B = 2 * nl * P;
    const int Npad = P * L;
    double *fwd = tab + kCoefHdr;                        // Npad x 2
    double *bwd = fwd + (int64_t)Npad * 2;               // Npad x 3
    double *spk = fwd + (int64_t)Npad * 5;
    double *krow = spk + (int64_t)P * 2 * nl * L;
    double *K = scratch + (int64_t)t * scratch_per;      // B x B
    double *Kinv = K + (int64_t)B * B;                   // B x B
    double *v = Kinv + (int64_t)B * B;                   // L
    double *facs = v + L;                                // Npad x 5 (l1, l2, u1, u2, 1/d)
    int bad = 0;

    // 1. partition-local banded LU without pivoting (Doolittle, nl <= 2)
    for (int p = 0; p < P; ++p) {
        double *F = facs + (int64_t)p * L * 5;
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
    for (int k = 0; k < Npad; ++k) {
        fwd[k * 2 + 0] = facs[k * 5 + 0];
        fwd[k * 2 + 1] = facs[k * 5 + 1];
        bwd[k * 3 + 0] = facs[k * 5 + 2];
        bwd[k * 3 + 1] = facs[k * 5 + 3];
        bwd[k * 3 + 2] = facs[k * 5 + 4];
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
                    if (s.periodic || (col >= 0 && col < Npad)) e = dl_entry(s, k, o);
                }
                v[i] = e;
            }
            local_solve(facs + (int64_t)p * L * 5, L, nl, v);
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
    // 5. end-value influence vectors of an iterated closure: the solution for
    //    a right side gamma at row 0 (left end value) and at row N - 1 (right),
    //    by the same partition algebra the line kernel runs; zero otherwise
    double *gv = krow + (int64_t)P * 2 * nl * B;         // [2][Npad]
    double *yb = facs + (int64_t)Npad * 5;               // B boundary entries
    double *gtmp = yb + B;                               // Npad
    for (int side = 0; side < 2; ++side) {
        double *g = gv + (int64_t)side * Npad;
        for (int k = 0; k < Npad; ++k) g[k] = 0.0;
        if (!s.ext || s.periodic) continue;
        g[side ? s.N - 1 : 0] = s.gamma;
        for (int p = 0; p < P; ++p) local_solve(facs + (int64_t)p * L * 5, L, nl, g + (int64_t)p * L);
        for (int p = 0; p < P; ++p)
            for (int tq = 0; tq < 2 * nl; ++tq) yb[p * 2 * nl + tq] = g[p * L + (tq < nl ? tq : L - 2 * nl + tq)];
        for (int k = 0; k < Npad; ++k) gtmp[k] = g[k];
        for (int p = 0; p < P; ++p) {
            for (int q = 0; q < 2 * nl; ++q) {
                double xq = 0.0;
                for (int b = 0; b < B; ++b) xq += krow[((int64_t)p * 2 * nl + q) * B + b] * yb[b];
                for (int i = 0; i < L; ++i) gtmp[p * L + i] -= xq * spk[((int64_t)p * 2 * nl + q) * L + i];
            }
        }
        for (int k = 0; k < Npad; ++k) g[k] = gtmp[k];
    }
    status[t] = bad;
}

// XCD (accelerator complex die) that runs each workgroup, one record per
// workgroup: the plan checks on it that every aligned group of kXCD
// consecutive workgroups is spread over all kXCD dies before it offers the
// XCD-interleaved per-item order.
__global__ void k_xcc_probe(int *__restrict__ out) {
    if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);   // HW_REG_XCC_ID
}

// Number of 32-bit words that differ between a and b (bitwise).
__global__ void k_count_diff(int64_t n, const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                             unsigned long long *__restrict__ cnt) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += a[i] != b[i];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

template <typename T>
__global__ void k_count_nonfinite(int64_t n, const T *__restrict__ x, unsigned long long *cnt) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += !isfinite(x[i]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// Registry of compiled line-kernel classes
// ---------------------------------------------------------------------------
extern const LineClass kLineClassesF64[] = { CFD_LINE_CLASSES(double, 0) };
extern const int kNumLineClassesF64 = (int)(sizeof(kLineClassesF64) / sizeof(kLineClassesF64[0]));

namespace {
// The classes of one precision: the plain table, then the extension table.
template <typename F>
void for_each_class(int f32, F &&fn) {
    const LineClass *tabs[2] = {f32 ? kLineClassesF32 : kLineClassesF64, f32 ? kLineClassesExtF32 : kLineClassesExtF64};
    const int ns[2] = {f32 ? kNumLineClassesF32 : kNumLineClassesF64,
                       f32 ? kNumLineClassesExtF32 : kNumLineClassesExtF64};
    for (int t = 0; t < 2; ++t)
        for (int i = 0; i < ns[t]; ++i) fn(tabs[t][i]);
}
}  // namespace

const LineClass *find_line_class(int f32, int nl, int nops, int par, int mi, int hw, int L, int ext, int wg) {
    const LineClass *best = nullptr;
    for_each_class(f32, [&](const LineClass &k) {
        if (k.nl != nl || k.nops != nops || k.par != par || k.mi < mi || k.hw < hw || k.ext != ext) return;
        if (k.wg != wg) return;
        bool hasL = false;
        for (int j = 0; j < k.nL; ++j) hasL |= (k.Ls[j] == L);
        if (!hasL) return;
        if (!best || (k.mi + k.hw) < (best->mi + best->hw) ||
            ((k.mi + k.hw) == (best->mi + best->hw) && k.nL < best->nL))
            best = &k;
    });
    return best;
}

int line_class_Ls(int f32, int nl, int nops, int par, int mi, int hw, int *Ls, int cap, int ext, int wg) {
    int cnt = 0;
    for_each_class(f32, [&](const LineClass &k) {
        if (k.nl != nl || k.nops != nops || k.par != par || k.mi < mi || k.hw < hw || k.ext != ext) return;
        if (wg && k.wg != wg) return;
        for (int j = 0; j < k.nL; ++j) {
            bool seen = false;
            for (int q = 0; q < cnt; ++q) seen |= (Ls[q] == k.Ls[j]);
            if (!seen && cnt < cap) Ls[cnt++] = k.Ls[j];
        }
    });
    return cnt;
}

hipError_t launch_lines(const void *fn, int wg, int grid, size_t lds, hipStream_t st, const WorkItem *items, int nitems,
                        const int *qoff, const PassDesc *passes, const void *tabs, const int64_t *taboff,
                        const void *in, void *out, const void *ev, const RkArgs *rk) {
    RkArgs r{};
    if (rk) r = *rk;
    void *args[] = {(void *)&items, (void *)&nitems, (void *)&qoff, (void *)&passes, (void *)&tabs,
                    (void *)&taboff, (void *)&in, (void *)&out, (void *)&ev, (void *)&r};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * wg), args, lds, st);
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

hipError_t launch_xcc_probe(int grid, int *out, hipStream_t st) {
    hipLaunchKernelGGL(k_xcc_probe, dim3(grid), dim3(64), 0, st, out);
    return hipGetLastError();
}

hipError_t launch_count_diff(int64_t nwords, const void *a, const void *b, unsigned long long *cnt, hipStream_t st) {
    int grid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (nwords + 255) / 256));
    hipLaunchKernelGGL(k_count_diff, dim3(grid), dim3(256), 0, st, nwords, (const uint32_t *)a, (const uint32_t *)b,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(int f32, int64_t n, const void *x, unsigned long long *cnt, hipStream_t st) {
    int grid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
    if (f32)
        hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(grid), dim3(256), 0, st, n, (const float *)x, cnt);
    else
        hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(grid), dim3(256), 0, st, n, (const double *)x, cnt);
    return hipGetLastError();
}

size_t tabspec_size() { return sizeof(TabSpec); }

void fill_tabspec(void *dst, int N, int P, int L, int nl, int nc, int periodic, const double *alpha5, int64_t off,
                  int ext, double cl_d0, double cl_up, double gamma) {
    TabSpec s;
    s.N = N; s.P = P; s.L = L; s.nl = nl; s.nc = nc; s.periodic = periodic;
    for (int i = 0; i < 2 * kMaxNL + 1; ++i) s.alpha[i] = alpha5[i];
    s.off = off;
    s.ext = ext; s.cl_d0 = cl_d0; s.cl_up = cl_up; s.gamma = gamma;
    *reinterpret_cast<TabSpec *>(dst) = s;
}

}  // namespace cfd
