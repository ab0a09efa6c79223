/*
 * Oracle line operator for compact finite differences (plain C, FP64).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU baseline.  It shares no code with the GPU library.
 *
 * What it computes (arXiv 2302.14858):
 *   Block closure, Eq. sch_cent_om (Sec. 2.4): on a line with N interior nodes
 *   k = 0..N-1 (k*_- = 0, k*_+ = N-1) and ng ghost nodes per side,
 *     - the nc rows nearest each end take the explicit closure stencil,
 *       f~_k = h^-d sum_m cbar_m f_{k+m};
 *     - every other row is an implicit interior row,
 *       sum_{|j|<=nl} alpha_j f~_{k+j} = h^-d sum_{|m|<=M} a_m f_{k+m},
 *       where f~ values on closure rows are known and moved to the right side;
 *     - the banded system left over is solved by Gaussian elimination without
 *       pivoting (the Thomas algorithm when nl = 1), as the paper's TDMA.
 *   Periodic lines (the periodic D of Sec. 2.2): every row is an interior row
 *   with indices taken modulo N; the cyclic system is solved by the
 *   Sherman-Morrison-Woodbury formula around the banded part.
 *
 * Right-end closure rows use the mirror image of the left ones:
 * cbar_right_j[m] = (-1)^d cbar_left_j[-m], the reflection rule of a centred
 * stencil for derivative degree d.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int d;          /* derivative degree d_r */
    double h;       /* grid spacing */
    int nl;         /* implicit half-width (0 explicit, 1 tri, 2 penta) */
    const double *alpha; /* 2nl+1 entries, alpha[nl] = 1 */
    int M;          /* interior RHS half-width */
    const double *a;     /* 2M+1 */
    int nc;         /* closure rows per end */
    int mc;         /* closure half-width */
    const double *cbar;  /* nc rows of 2mc+1 */
} orc_scheme;

/* Gaussian elimination without pivoting on the banded Toeplitz matrix
 * with diagonals alpha[-nl..nl], size n, for one right-hand side (in place).
 * band is scratch of n*(2nl+1) doubles. */
static void band_solve(int n, int nl, const double *alpha, double *band, double *rhs)
{
    int w = 2 * nl + 1;
    for (int i = 0; i < n; ++i)
        for (int j = -nl; j <= nl; ++j)
            band[i * w + (j + nl)] = (i + j >= 0 && i + j < n) ? alpha[j + nl] : 0.0;
    /* forward elimination: row i removes its entries left of the diagonal */
    for (int i = 0; i < n; ++i) {
        for (int j = -nl; j < 0; ++j) {
            int p = i + j;              /* pivot row */
            if (p < 0) continue;
            double f = band[i * w + (j + nl)] / band[p * w + nl];
            if (f == 0.0) continue;
            /* row_i -= f * row_p over columns p..p+nl */
            for (int c = 0; c <= nl; ++c) {
                int col = p + c;        /* absolute column */
                int oi = col - i;       /* offset within row i */
                if (oi < -nl || oi > nl) continue;
                band[i * w + (oi + nl)] -= f * band[p * w + (c + nl)];
            }
            rhs[i] -= f * rhs[p];
        }
    }
    /* back substitution */
    for (int i = n - 1; i >= 0; --i) {
        double s = rhs[i];
        for (int j = 1; j <= nl; ++j)
            if (i + j < n) s -= band[i * w + (j + nl)] * rhs[i + j];
        rhs[i] = s / band[i * w + nl];
    }
}

/* Dense R x R solve with partial pivoting (R <= 8). */
static void small_solve(int R, double *A, double *b)
{
    for (int c = 0; c < R; ++c) {
        int p = c;
        for (int r = c + 1; r < R; ++r)
            if (fabs(A[r * R + c]) > fabs(A[p * R + c])) p = r;
        if (p != c) {
            for (int k = 0; k < R; ++k) { double t = A[c * R + k]; A[c * R + k] = A[p * R + k]; A[p * R + k] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < R; ++r) {
            double f = A[r * R + c] / A[c * R + c];
            for (int k = c; k < R; ++k) A[r * R + k] -= f * A[c * R + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = R - 1; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < R; ++k) s -= A[c * R + k] * b[k];
        b[c] = s / A[c * R + c];
    }
}

static double hpow(double h, int d)
{
    double v = 1.0;
    for (int i = 0; i < d; ++i) v *= h;
    return v;
}

/* Work space needed per line (doubles). */
static size_t line_work(int N, int nl)
{
    size_t w = 2 * (size_t)nl + 1;
    size_t R = 2 * (size_t)nl;
    return (size_t)N * w + (size_t)N * (R + 2) + R * R + 4 * R + 16;
}

/* One block line.  g points at the first ghost node: g[ng + k] is node k.
 * x receives N outputs (already multiplied by h^-d). */
static void line_closure(const orc_scheme *s, int N, int ng, const double *g, double *x, double *work)
{
    const double hinv = 1.0 / hpow(s->h, s->d);
    const int nc = s->nl > 0 ? s->nc : 0;
    const double sgn = (s->d % 2) ? -1.0 : 1.0;
    const int w = 2 * s->mc + 1;

    for (int j = 0; j < nc; ++j) {
        const double *c = s->cbar + (size_t)j * w;
        double acc = 0.0, accr = 0.0;
        for (int m = -s->mc; m <= s->mc; ++m) {
            acc += c[m + s->mc] * g[ng + j + m];
            accr += sgn * c[-m + s->mc] * g[ng + (N - 1 - j) + m];
        }
        x[j] = hinv * acc;
        x[N - 1 - j] = hinv * accr;
    }
    int n = N - 2 * nc;
    double *r = work;                       /* n */
    double *band = work + N;                /* n*(2nl+1) */
    for (int i = 0; i < n; ++i) {
        int k = nc + i;
        double acc = 0.0;
        for (int m = -s->M; m <= s->M; ++m) acc += s->a[m + s->M] * g[ng + k + m];
        double v = hinv * acc;
        for (int j = -s->nl; j <= s->nl; ++j) {
            int kk = k + j;
            if (j != 0 && (kk < nc || kk > N - 1 - nc)) v -= s->alpha[j + s->nl] * x[kk];
        }
        r[i] = v;
    }
    if (s->nl > 0) band_solve(n, s->nl, s->alpha, band, r);
    for (int i = 0; i < n; ++i) x[nc + i] = r[i];
}

/* One periodic line: node k reads g[ng + ((k+m) mod N)]. */
static void line_periodic(const orc_scheme *s, int N, int ng, const double *g, double *x, double *work)
{
    const double hinv = 1.0 / hpow(s->h, s->d);
    const int nl = s->nl;
    for (int k = 0; k < N; ++k) {
        double acc = 0.0;
        for (int m = -s->M; m <= s->M; ++m) {
            int kk = ((k + m) % N + N) % N;
            acc += s->a[m + s->M] * g[ng + kk];
        }
        x[k] = hinv * acc;
    }
    if (nl == 0) return;
    /* A = A_band + U V^T, the wrap-around entries of rows 0..nl-1 and N-nl..N-1 */
    const int R = 2 * nl;
    double *band = work;                    /* N*(2nl+1) */
    double *Z = band + (size_t)N * (2 * nl + 1); /* R columns of length N */
    double *S = Z + (size_t)N * R;          /* R*R */
    double *vy = S + R * R;                 /* R */
    int rows[8];
    for (int t = 0; t < nl; ++t) { rows[t] = t; rows[nl + t] = N - nl + t; }
    /* V: corner coefficients of each such row */
    double V[8][8 * 2];
    int Vcol[8][8];
    int Vn[8];
    for (int q = 0; q < R; ++q) {
        int i = rows[q];
        Vn[q] = 0;
        for (int j = -nl; j <= nl; ++j) {
            int col = i + j;
            if (col < 0 || col >= N) {
                Vcol[q][Vn[q]] = (col % N + N) % N;
                V[q][Vn[q]] = s->alpha[j + nl];
                Vn[q]++;
            }
        }
    }
    for (int q = 0; q < R; ++q) {
        double *z = Z + (size_t)q * N;
        memset(z, 0, sizeof(double) * N);
        z[rows[q]] = 1.0;
        band_solve(N, nl, s->alpha, band, z);
    }
    band_solve(N, nl, s->alpha, band, x);  /* y */
    for (int p = 0; p < R; ++p) {
        double acc = 0.0;
        for (int t = 0; t < Vn[p]; ++t) acc += V[p][t] * x[Vcol[p][t]];
        vy[p] = acc;
        for (int q = 0; q < R; ++q) {
            double sz = 0.0;
            for (int t = 0; t < Vn[p]; ++t) sz += V[p][t] * Z[(size_t)q * N + Vcol[p][t]];
            S[p * R + q] = (p == q ? 1.0 : 0.0) + sz;
        }
    }
    small_solve(R, S, vy);
    for (int k = 0; k < N; ++k) {
        double c = 0.0;
        for (int q = 0; q < R; ++q) c += Z[(size_t)q * N + k] * vy[q];
        x[k] -= c;
    }
}

/* Exported: one line.  g has N + 2*ng entries (ghosts included). */
int orc_line(int N, int ng, int periodic,
             int d, double h, int nl, const double *alpha, int M, const double *a,
             int nc, int mc, const double *cbar,
             const double *g, double *x)
{
    orc_scheme s = {d, h, nl, alpha, M, a, nc, mc, cbar};
    if (N < 1) return 1;
    double *work = (double *)malloc(sizeof(double) * line_work(N, nl));
    if (!work) return 2;
    if (periodic) line_periodic(&s, N, ng, g, x, work);
    else line_closure(&s, N, ng, g, x, work);
    free(work);
    return 0;
}

/* Exported: every line of one block-field along direction dir (0=x,1=y,2=z).
 * in : [z][y][x] with extents (n+2ng) per dimension, ghosts included.
 * out: [z][y][x] interior only.
 * periodic: the block wraps in direction dir (its ghosts are not read). */
int orc_block_dir(int nx, int ny, int nz, int ng, int dir, int periodic,
                  int d, double h, int nl, const double *alpha, int M, const double *a,
                  int nc, int mc, const double *cbar,
                  const double *in, double *out, int nthreads)
{
    orc_scheme s = {d, h, nl, alpha, M, a, nc, mc, cbar};
    const long PX = nx + 2L * ng, PY = ny + 2L * ng;
    const int n[3] = {nx, ny, nz};
    const int N = n[dir];
    const int u = dir == 0 ? 1 : 0;        /* the two other directions */
    const int v = dir == 2 ? 1 : 2;
    const long nlines = (long)n[u] * n[v];
    const long gstride[3] = {1, PX, PX * PY};
    const long ostride[3] = {1, nx, (long)nx * ny};
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *g = (double *)malloc(sizeof(double) * (N + 2 * ng));
        double *x = (double *)malloc(sizeof(double) * N);
        double *work = (double *)malloc(sizeof(double) * line_work(N, nl));
        if (!g || !x || !work) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(static)
            for (long l = 0; l < nlines; ++l) {
                int c[3];
                c[u] = (int)(l % n[u]);
                c[v] = (int)(l / n[u]);
                c[dir] = 0;
                long gbase = (c[2] + ng) * gstride[2] + (c[1] + ng) * gstride[1] + (c[0] + ng) * gstride[0];
                long obase = c[2] * ostride[2] + c[1] * ostride[1] + c[0] * ostride[0];
                for (int k = -ng; k < N + ng; ++k) g[k + ng] = in[gbase + k * gstride[dir]];
                if (periodic) line_periodic(&s, N, ng, g, x, work);
                else line_closure(&s, N, ng, g, x, work);
                for (int k = 0; k < N; ++k) out[obase + k * ostride[dir]] = x[k];
            }
        }
        free(g); free(x); free(work);
    }
    return bad ? 2 : 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
