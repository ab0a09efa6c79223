// Scheme construction for the compact finite-difference library, on the host
// in binary128 (__float128) arithmetic.
//
// Follows arXiv 2302.14858, Sec. 2 and 2.4:
//  * centred schemes of Eq. mdAnsatz with d_I = (0): alpha^(d) of half-width nl
//    (alpha^(d)_0 = 1) and alpha^(0) of half-width m;
//  * Taylor matching (Eq. Tcons) up to the formal order;
//  * when coefficients remain free, minimisation of the spectral error of
//    Eqs. sp_error / optfunc with the cut-off weight of Eq. gammacut;
//  * explicit closures of Sec. 2.4: Taylor conditions, plus, for the matched
//    variant, the lowest error constant of the interior scheme
//    (Eq. errrelmodwavcent) imposed on the closure (the odd power that follows
//    vanishes by symmetry for a centred stencil).
//
// Centred schemes are parametrised by their symmetry from the start: alpha^(d)
// is symmetric, alpha^(0) is antisymmetric for odd d and symmetric for even d.
// The spectral error of such a scheme is a real function of eta, and the
// constrained quadratic minimisation is solved in the null space of the Taylor
// conditions with Gauss-Legendre quadrature on [0, eta_c].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cfd_internal.h"

namespace cfd {
namespace {

typedef __float128 q;

q qabs(q x) { return x < 0 ? -x : x; }

// pi to 36 significant digits
const q kPi = (q)3.14159265358979323846264338327950288Q;

// sin / cos by reduction to [-pi, pi] and the Taylor series (enough terms for
// binary128 on that interval).
void qsincos(q x, q &s, q &c) {
    q twopi = 2 * kPi;
    q k = (q)(long long)(x / twopi + (x >= 0 ? (q)0.5 : (q)-0.5));
    x -= k * twopi;
    q term = x, sum_s = x;
    q termc = 1, sum_c = 1;
    q x2 = x * x;
    for (int n = 1; n < 60; ++n) {
        term *= -x2 / ((2 * n) * (2 * n + 1));
        termc *= -x2 / ((2 * n - 1) * (2 * n));
        sum_s += term;
        sum_c += termc;
    }
    s = sum_s;
    c = sum_c;
}

q qpow_int(q x, int p) {
    q r = 1;
    for (int i = 0; i < p; ++i) r *= x;
    return r;
}

q qfact(int n) {
    q r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// Gauss-Legendre nodes and weights on [a, b] (Newton on P_n).
void gauss_legendre(int n, q a, q b, std::vector<q> &x, std::vector<q> &w) {
    x.assign(n, 0);
    w.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        q z = (q)std::cos(M_PI * (i + 0.75) / (n + 0.5));
        q pp = 0;
        for (int it = 0; it < 100; ++it) {
            q p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                q p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            pp = n * (z * p1 - p0) / (z * z - 1);
            q dz = p1 / pp;
            z -= dz;
            if (qabs(dz) < (q)1e-33Q) break;
        }
        x[i] = (a + b) / 2 + (b - a) / 2 * z;
        w[i] = (b - a) / ((1 - z * z) * pp * pp);
    }
}

// Dense solve with partial pivoting; A is n x n row-major.  false if singular.
bool qsolve(int n, std::vector<q> A, std::vector<q> &b) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (qabs(A[r * n + c]) > qabs(A[p * n + c])) p = r;
        if (qabs(A[p * n + c]) < (q)1e-60Q) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
            std::swap(b[c], b[p]);
        }
        for (int r = c + 1; r < n; ++r) {
            q f = A[r * n + c] / A[c * n + c];
            if (f == 0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        q s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
    return true;
}

// Unknowns of a centred scheme: alpha_1..alpha_nl, then the RHS parameters
// b_{m0}..b_m (m0 = 1 for odd d, 0 for even d).  a_{+-k} = (+-1)^d b_k.
struct Centred {
    int d, nl, m;
    int m0() const { return (d % 2) ? 1 : 0; }
    int nunk() const { return nl + (m - m0() + 1); }
};

// Taylor row l of Eq. Tcons for a centred scheme, as coefficients of the
// unknowns plus a constant (the alpha_0 = 1 contribution):
//   sum_k a_k k^l / l!  -  sum_j alpha_j j^(l-d)/(l-d)!  = 0.
void taylor_row(const Centred &c, int l, std::vector<q> &row, q &cst) {
    row.assign(c.nunk(), 0);
    cst = 0;
    // alpha part (symmetric): j = 0 gives 1 when l == d; j = +-1.. gives 2 j^(l-d)/(l-d)! for even l-d
    if (l >= c.d) {
        int p = l - c.d;
        if (p == 0) cst -= 1;  // alpha_0 = 1 moved to the constant (with the minus sign)
        if (p % 2 == 0)
            for (int j = 1; j <= c.nl; ++j) row[j - 1] -= 2 * qpow_int(j, p) / qfact(p);
    }
    // RHS part: sum_k a_k k^l with a antisymmetric (odd d) or symmetric (even d)
    for (int k = c.m0(); k <= c.m; ++k) {
        q v;
        if (k == 0) v = (l == 0) ? 1 : 0;
        else if ((c.d % 2) == 1) v = (l % 2 == 1) ? 2 * qpow_int(k, l) : 0;
        else v = (l % 2 == 0) ? 2 * qpow_int(k, l) : 0;
        row[c.nl + (k - c.m0())] += v / qfact(l);
    }
}

bool row_trivial(const std::vector<q> &row, q cst) {
    if (cst != 0) return false;
    for (q v : row)
        if (v != 0) return false;
    return true;
}

// Real spectral error e(eta) = g(eta).u + g0(eta) of a centred scheme
// (Eq. sp_error up to a unit factor i for odd d).
void spectral_basis(const Centred &c, q eta, std::vector<q> &g, q &g0) {
    g.assign(c.nunk(), 0);
    if (c.d == 1) {
        // e~ = i [ 2 sum b_k sin(k eta) - eta (1 + 2 sum alpha_j cos(j eta)) ]
        g0 = -eta;
        for (int j = 1; j <= c.nl; ++j) {
            q s, co;
            qsincos(j * eta, s, co);
            g[j - 1] = -2 * eta * co;
        }
        for (int k = 1; k <= c.m; ++k) {
            q s, co;
            qsincos(k * eta, s, co);
            g[c.nl + k - 1] = 2 * s;
        }
    } else {
        // e~ = b_0 + 2 sum b_k cos(k eta) + eta^2 (1 + 2 sum alpha_j cos(j eta))
        g0 = eta * eta;
        for (int j = 1; j <= c.nl; ++j) {
            q s, co;
            qsincos(j * eta, s, co);
            g[j - 1] = 2 * eta * eta * co;
        }
        for (int k = 0; k <= c.m; ++k) {
            q s, co;
            qsincos(k * eta, s, co);
            g[c.nl + k] = (k == 0) ? (q)1 : 2 * co;
        }
    }
}

// Solve the (possibly underdetermined) constraint set C u = rhs by
// Gauss-Jordan with full pivoting; returns a particular solution and a basis
// of the null space.  false if inconsistent.
bool null_space(int nr, int n, std::vector<q> C, std::vector<q> rhs, std::vector<q> &up,
                std::vector<std::vector<q>> &Z) {
    std::vector<int> pivcol;
    int r = 0;
    std::vector<bool> used(n, false);
    for (int c = 0; c < n && r < nr; ++c) {
        int p = -1;
        q best = 0;
        for (int i = r; i < nr; ++i)
            if (qabs(C[i * n + c]) > best) { best = qabs(C[i * n + c]); p = i; }
        if (p < 0 || best < (q)1e-40Q) continue;
        for (int k = 0; k < n; ++k) std::swap(C[r * n + k], C[p * n + k]);
        std::swap(rhs[r], rhs[p]);
        q pv = C[r * n + c];
        for (int k = 0; k < n; ++k) C[r * n + k] /= pv;
        rhs[r] /= pv;
        for (int i = 0; i < nr; ++i) {
            if (i == r) continue;
            q f = C[i * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; ++k) C[i * n + k] -= f * C[r * n + k];
            rhs[i] -= f * rhs[r];
        }
        pivcol.push_back(c);
        used[c] = true;
        ++r;
    }
    for (int i = r; i < nr; ++i)
        if (qabs(rhs[i]) > (q)1e-28Q) return false;
    up.assign(n, 0);
    for (int i = 0; i < r; ++i) up[pivcol[i]] = rhs[i];
    Z.clear();
    for (int f = 0; f < n; ++f) {
        if (used[f]) continue;
        std::vector<q> z(n, 0);
        z[f] = 1;
        for (int i = 0; i < r; ++i) z[pivcol[i]] = -C[i * n + f];
        Z.push_back(z);
    }
    return true;
}

q dot(const std::vector<q> &a, const std::vector<q> &b) {
    q s = 0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------

cfd_status design_centred(int d, int order, int nl, int m, double eta_c, int closure_mc,
                          int matched, Scheme &out, std::string &err) {
    if (d < 1 || d > 2 || order < 2 || order % 2 || nl < 0 || nl > kMaxNL || m < 1 ||
        m > kMaxHalf || closure_mc < 0 || closure_mc > kMaxHalf) {
        err = "scheme design: unsupported d/order/nl/m/closure size";
        return CFD_EINVAL;
    }
    Centred c{d, nl, m};
    const int n = c.nunk();
    // Taylor rows l = 0 .. order + d - 1 that are not identically zero by symmetry
    std::vector<q> C, rhs;
    int nr = 0;
    for (int l = 0; l < order + d; ++l) {
        std::vector<q> row;
        q cst;
        taylor_row(c, l, row, cst);
        if (row_trivial(row, cst)) continue;
        C.insert(C.end(), row.begin(), row.end());
        rhs.push_back(-cst);
        ++nr;
    }
    std::vector<q> up;
    std::vector<std::vector<q>> Z;
    if (!null_space(nr, n, C, rhs, up, Z)) {
        err = "scheme design: Taylor conditions are inconsistent";
        return CFD_ESINGULAR;
    }
    std::vector<q> u = up;
    if (!Z.empty()) {
        if (!(eta_c > 0) || eta_c > M_PI + 1e-12) {
            err = "scheme design: free coefficients need 0 < eta_c <= pi";
            return CFD_EINVAL;
        }
        // eta_c given as double; recognise 4pi/5 and pi exactly
        q ec = (q)eta_c;
        if (std::fabs(eta_c - 4 * M_PI / 5) < 1e-12) ec = 4 * kPi / 5;
        if (std::fabs(eta_c - M_PI) < 1e-12) ec = kPi;
        std::vector<q> xs, ws;
        gauss_legendre(48, 0, ec, xs, ws);
        const int nf = (int)Z.size();
        std::vector<q> H(nf * nf, 0), h(nf, 0);
        for (size_t t = 0; t < xs.size(); ++t) {
            std::vector<q> g;
            q g0;
            spectral_basis(c, xs[t], g, g0);
            q e0 = dot(g, up) + g0;
            std::vector<q> ez(nf);
            for (int i = 0; i < nf; ++i) ez[i] = dot(g, Z[i]);
            for (int i = 0; i < nf; ++i) {
                h[i] -= ws[t] * ez[i] * e0;
                for (int j = 0; j < nf; ++j) H[i * nf + j] += ws[t] * ez[i] * ez[j];
            }
        }
        if (!qsolve(nf, H, h)) {
            err = "scheme design: spectral objective is degenerate";
            return CFD_ESINGULAR;
        }
        for (int i = 0; i < nf; ++i)
            for (int k = 0; k < n; ++k) u[k] += h[i] * Z[i][k];
    }
    Scheme s;
    s.d = d;
    s.order = order;
    s.nl = nl;
    s.m = m;
    s.lhs[kMaxNL] = 1.0;
    q dn0 = 1;  // alpha . E at eta = 0
    for (int j = 1; j <= nl; ++j) {
        s.lhs[kMaxNL + j] = s.lhs[kMaxNL - j] = (double)u[j - 1];
        dn0 += 2 * u[j - 1];
    }
    std::vector<q> a(2 * kMaxHalf + 1, 0);
    for (int k = c.m0(); k <= m; ++k) {
        q b = u[nl + k - c.m0()];
        a[kMaxHalf + k] = b;
        a[kMaxHalf - k] = (d % 2 && k > 0) ? -b : b;
    }
    for (int k = -kMaxHalf; k <= kMaxHalf; ++k) s.rhs[kMaxHalf + k] = (double)a[kMaxHalf + k];

    // Error constant of the interior scheme: T_{q+d} / (alpha . E)(0), with
    // T_l the Taylor residual of row l (the eta^q coefficient of eps up to i^q).
    q Tqd = 0;
    {
        int l = order + d;
        for (int k = -m; k <= m; ++k) Tqd += a[kMaxHalf + k] * qpow_int(k, l) / qfact(l);
        // alpha part
        for (int j = -nl; j <= nl; ++j) {
            q al = (j == 0) ? (q)1 : u[std::abs(j) - 1];
            Tqd -= al * qpow_int(j, order) / qfact(order);
        }
    }

    if (nl > 0 && closure_mc > 0) {
        // closure unknowns: c_1..c_mc (odd d) or c_0..c_mc (even d)
        Centred cc{d, 0, closure_mc};
        const int ncu = cc.nunk();
        std::vector<q> CC, rr;
        int nrc = 0;
        for (int l = 0; l < order + d; ++l) {
            std::vector<q> row;
            q cst;
            taylor_row(cc, l, row, cst);
            if (row_trivial(row, cst)) continue;
            CC.insert(CC.end(), row.begin(), row.end());
            rr.push_back(-cst);
            ++nrc;
        }
        if (matched) {
            std::vector<q> row;
            q cst;
            taylor_row(cc, order + d, row, cst);  // explicit: cst == 0 for l > d
            CC.insert(CC.end(), row.begin(), row.end());
            rr.push_back(Tqd / dn0);
            ++nrc;
        }
        if (nrc != ncu) {
            err = "scheme design: closure half-width does not match the number of closure conditions";
            return CFD_EINVAL;
        }
        std::vector<q> sol = rr;
        if (!qsolve(ncu, CC, sol)) {
            err = "scheme design: closure conditions are singular";
            return CFD_ESINGULAR;
        }
        double row[2 * kMaxHalf + 1] = {0};
        for (int k = cc.m0(); k <= closure_mc; ++k) {
            q b = sol[k - cc.m0()];
            row[kMaxHalf + k] = (double)b;
            row[kMaxHalf - k] = (double)((d % 2 && k > 0) ? -b : b);
        }
        s.nc = nl;
        s.mc = closure_mc;
        for (int j = 0; j < nl; ++j) std::memcpy(s.cl[j], row, sizeof(row));
    }
    cfd_status sst = check_symbol(s, err);
    if (sst != CFD_OK) {
        err = "scheme design: " + err;
        return sst;
    }
    out = s;
    return CFD_OK;
}

// ---------------------------------------------------------------------------
// Fully determined schemes of the multi-derivative ansatz (Eq. mdAnsatz with
// any sample classes d_I, Eq. Tcons), e.g. the biased schemes of Eq.
// defChenSchemes or the worked example of Sec. 2.  Unknowns: alpha^(dr) on
// -L..R with alpha^(dr)_0 = 1, then each class on -Lk..Rk.  Taylor row l:
//   sum_c sum_n a^(dc)_n n^(l-dc)/(l-dc)!  -  sum_n alpha^(dr)_n n^(l-dr)/(l-dr)!  = 0.
// As many rows as unknowns (after the normalisation) are imposed; the order is
// the first violated row minus dr.
// ---------------------------------------------------------------------------
namespace {

struct Ansatz {
    int dr, L, R;
    std::vector<int> dI, Lk, Rk;
    int nunk() const {
        int n = L + R + 1;
        for (size_t c = 0; c < dI.size(); ++c) n += Lk[c] + Rk[c] + 1;
        return n;
    }
};

void ansatz_row(const Ansatz &a, int l, std::vector<q> &row) {
    row.assign(a.nunk(), 0);
    int col = 0;
    for (int n = -a.L; n <= a.R; ++n, ++col)
        if (l >= a.dr) row[col] = -qpow_int(n, l - a.dr) / qfact(l - a.dr);   // 0^0 = 1
    for (size_t c = 0; c < a.dI.size(); ++c)
        for (int n = -a.Lk[c]; n <= a.Rk[c]; ++n, ++col)
            if (l >= a.dI[c]) row[col] = qpow_int(n, l - a.dI[c]) / qfact(l - a.dI[c]);
}

bool ansatz_solve(const Ansatz &a, std::vector<q> &x, int &order) {
    const int n = a.nunk();
    std::vector<q> A((size_t)n * n, 0), b(n, 0);
    A[a.L] = 1;   // alpha^(dr)_0 = 1
    b[0] = 1;
    for (int l = 0; l < n - 1; ++l) {
        std::vector<q> row;
        ansatz_row(a, l, row);
        for (int k = 0; k < n; ++k) A[(size_t)(l + 1) * n + k] = row[k];
    }
    if (!qsolve(n, A, b)) return false;
    x = b;
    int l = n - 1;
    for (;; ++l) {
        std::vector<q> row;
        ansatz_row(a, l, row);
        q r = 0, sc = 0;
        for (int k = 0; k < n; ++k) {
            r += row[k] * x[k];
            sc += qabs(row[k] * x[k]);
        }
        if (qabs(r) > (q)1e-28Q * (sc + 1)) break;
        if (l > 64) break;
    }
    order = l - a.dr;
    return true;
}

// One biased first-degree scheme in working precision: alpha x_{k-1} + x_k =
// sum_m a_m f_{k+m} (+ a2 dx^2 f''_k for U).
struct BiasedQ {
    q alpha = 0, a2 = 0;
    q a[2 * 8 + 1] = {0};     // offsets -8..8
    int order = 0;
    q at(int m) const { return (m < -8 || m > 8) ? (q)0 : a[m + 8]; }
};

bool ucd_scheme(char kind, int M, BiasedQ &s) {
    Ansatz an{1, 1, 0, {0}, {M}, {M}};
    if (kind == 'U') {
        an.dI.push_back(2);
        an.Lk.push_back(0);
        an.Rk.push_back(0);
    }
    std::vector<q> x;
    if (!ansatz_solve(an, x, s.order)) return false;
    s.alpha = x[0];
    for (int m = -M; m <= M; ++m) s.a[m + 8] = x[2 + m + M];
    s.a2 = (kind == 'U') ? x[2 + 2 * M + 1] : (q)0;
    return true;
}

// Taylor residual of row l of a biased scheme (no f'' term):
//   T_l = sum_m a_m m^l / l!  -  sum_j alpha_j j^(l-1)/(l-1)!.
q biased_residual(const BiasedQ &s, int l) {
    q t = 0;
    for (int m = -8; m <= 8; ++m)
        if (s.at(m) != 0) t += s.at(m) * qpow_int(m, l) / qfact(l);
    if (l >= 1) {
        t -= qpow_int(0, l - 1) / qfact(l - 1);                  // alpha_0 = 1
        t -= s.alpha * qpow_int(-1, l - 1) / qfact(l - 1);       // alpha_{-1}
    }
    return t;
}

}  // namespace

cfd_status taylor_scheme(int dr, int L, int R, int nclass, const int *dI, const int *Lk, const int *Rk,
                         std::vector<double> &coef, int &order, std::string &err) {
    if (dr < 0 || L < 0 || R < 0 || L + R > 16 || nclass < 1 || nclass > 4 || !dI || !Lk || !Rk) {
        err = "Taylor scheme: bad extents";
        return CFD_EINVAL;
    }
    Ansatz an{dr, L, R, {}, {}, {}};
    for (int c = 0; c < nclass; ++c) {
        if (dI[c] < 0 || Lk[c] < 0 || Rk[c] < 0 || Lk[c] + Rk[c] > 16) {
            err = "Taylor scheme: bad sample class";
            return CFD_EINVAL;
        }
        an.dI.push_back(dI[c]);
        an.Lk.push_back(Lk[c]);
        an.Rk.push_back(Rk[c]);
    }
    std::vector<q> x;
    if (!ansatz_solve(an, x, order)) {
        err = "Taylor scheme: the conditions are singular for these extents";
        return CFD_ESINGULAR;
    }
    coef.assign(x.size(), 0.0);
    for (size_t i = 0; i < x.size(); ++i) coef[i] = (double)x[i];
    return CFD_OK;
}

// Biased schemes of Sec. ssec:domdec_drp.
//  V_M (family 'V'): Eq. defChenSchemes with alpha^(2)_0 = 0, order 2M+1.
//  X_M (family 'X'): lambda U_M + (1 - lambda) V_{M+1} (Eq. LCslowfast) with
//    the f'' sample of U_M replaced by the explicit (2)E_{M+2}; order 2M+2.
//  W_M (family 'W'): the same combination keeping a2 dx^2 f''_k, with f'' the
//    compact centred (2)P1_M solved on the line with its matched explicit
//    closure (Tab. ccuw_deg_one_col); order 2M+2.  At k*_+ that f'' is the
//    closure's explicit value, so the row there is the interior row with the
//    closure stencil in place of f'' (the printed Wtilde); the closure at
//    k*_- is built, as below, from that explicit row.
// Closure at k*_-: the mirror image of the scheme plus xi dx^q (alpha^(1) .
// f^(q)) over its two implicit nodes, f^(q) from the centred (q)E_{q/2}
// (binomial differences, Tab. diss_scheme), q the first even order above the
// formal order.  xi matches the lowest imaginary term of the interior
// wavenumber error (Eqs. ucd_slow_closure_chi, ucd_fast_closure_chi).  With
// z = i eta, B(z)/A(z) = z + S(z) where S = T/A is the quotient of the
// Taylor-residual series T(z) = sum_l T_l z^l by A(z) = sum_k z^k sum_j
// alpha_j j^k/k!; then Im eta~ = -(-1)^(q/2) s_q eta^q + ..., the mirror
// flips its sign and the correction adds -xi (2 cos eta - 2)^(q/2), so
// xi = 2 s_q.
cfd_status design_biased(char family, int M, double lambda, int bias, Scheme &out, std::string &err) {
    if (bias < -1 || bias > 2) {
        err = "biased scheme: bias must be -1, +1, 0 (upwind pair) or 2 (symmetrised)";
        return CFD_EINVAL;
    }
    BiasedQ s;
    if (family == 'U') {
        if (M < 1 || M > 4) {
            err = "biased scheme: U_M needs 1 <= M <= 4";
            return CFD_EUNSUPPORTED;
        }
        if (!ucd_scheme('U', M, s)) {
            err = "biased scheme: singular Taylor system";
            return CFD_ESINGULAR;
        }
    } else if (family == 'V') {
        if (M < 1 || M > 4) {
            err = "biased scheme: V_M needs 1 <= M <= 4";
            return CFD_EUNSUPPORTED;
        }
        if (!ucd_scheme('V', M, s)) {
            err = "biased scheme: singular Taylor system";
            return CFD_ESINGULAR;
        }
    } else if (family == 'X') {
        if (M < 1 || M > 3) {
            err = "biased scheme: X_M needs 1 <= M <= 3";
            return CFD_EUNSUPPORTED;
        }
        // sigma printed with the X_M schemes (Tab. ccux_deg_one_col)
        static const q kLam[4] = {0, (q)37 / 100, (q)86 / 100, (q)146 / 100};
        const q lam = (lambda > 0) ? (q)lambda : kLam[M];
        BiasedQ u, v;
        if (!ucd_scheme('U', M, u) || !ucd_scheme('V', M + 1, v)) {
            err = "biased scheme: singular Taylor system";
            return CFD_ESINGULAR;
        }
        // (2)E_{M+2}: centred explicit second derivative
        Ansatz e2{2, 0, 0, {0}, {M + 2}, {M + 2}};
        std::vector<q> x;
        int o2 = 0;
        if (!ansatz_solve(e2, x, o2)) {
            err = "biased scheme: singular Taylor system";
            return CFD_ESINGULAR;
        }
        s.alpha = lam * u.alpha + (1 - lam) * v.alpha;
        for (int m = -8; m <= 8; ++m) {
            q e = (m >= -(M + 2) && m <= M + 2) ? x[1 + m + M + 2] : (q)0;
            s.a[m + 8] = lam * u.at(m) + (1 - lam) * v.at(m) + lam * u.a2 * e;
        }
        s.order = 2 * M + 2;
        // formal order check: rows 0..order vanish
        for (int l = 0; l <= s.order; ++l)
            if (qabs(biased_residual(s, l)) > (q)1e-28Q) {
                err = "biased scheme: combination lost its formal order";
                return CFD_ESINGULAR;
            }
    } else if (family == 'W') {
        if (M < 1 || M > 3) {
            err = "biased scheme: W_M needs 1 <= M <= 3";
            return CFD_EUNSUPPORTED;
        }
        // sigma printed with the W_M schemes (Tab. ccuw_deg_one_col)
        static const q kLamW[4] = {0, (q)38 / 100, (q)71 / 100, (q)95 / 100};
        const q lam = (lambda > 0) ? (q)lambda : kLamW[M];
        BiasedQ u, v;
        if (!ucd_scheme('U', M, u) || !ucd_scheme('V', M + 1, v)) {
            err = "biased scheme: singular Taylor system";
            return CFD_ESINGULAR;
        }
        s.alpha = lam * u.alpha + (1 - lam) * v.alpha;
        for (int m = -8; m <= 8; ++m) s.a[m + 8] = lam * u.at(m) + (1 - lam) * v.at(m);
        s.a2 = lam * u.a2;
        s.order = 2 * M + 2;
        for (int l = 0; l <= s.order; ++l)
            if (qabs(biased_residual(s, l) + (l == 2 ? s.a2 : (q)0)) > (q)1e-28Q) {
                err = "biased scheme: combination lost its formal order";
                return CFD_ESINGULAR;
            }
    } else {
        err = "biased scheme: unknown family (U, V, X or W)";
        return CFD_EINVAL;
    }
    // the row the closure is built from: the scheme itself, or for W the row
    // with f'' taken from the explicit closure of (2)P1_M
    BiasedQ sx = s;
    if (family == 'W') {
        Scheme p2;
        cfd_status pst = design_centred(2, 2 * M + 2, 1, M, 0.0, M + 2, true, p2, err);
        if (pst != CFD_OK) return pst;
        for (int m = -(M + 2); m <= M + 2; ++m) sx.a[m + 8] += s.a2 * (q)p2.cl[0][kMaxHalf + m];
        sx.a2 = 0;
    }
    const int p = s.order;
    const int qo = p + 2 - (p % 2);
    // S = T / A as power series in z up to z^qo
    std::vector<q> T(qo + 1), Am(qo + 1), S(qo + 1);
    for (int l = 0; l <= qo; ++l) T[l] = biased_residual(sx, l) + (l == 2 ? sx.a2 : (q)0);
    for (int k = 0; k <= qo; ++k) Am[k] = (k == 0 ? (q)1 : (q)0) + s.alpha * qpow_int(-1, k) / qfact(k);
    for (int n = 0; n <= qo; ++n) {
        q acc = T[n];
        for (int k = 1; k <= n; ++k) acc -= Am[k] * S[n - k];
        S[n] = acc / Am[0];
    }
    const q xi = 2 * S[qo];
    // closure at k*_-: mirror (alpha on the next node, stencil -a_{-m}) plus
    // xi sum_{j=0,1} w_j E_q(m - j), w = (1, alpha)
    const int h = qo / 2;
    q c[2 * 8 + 2] = {0};   // offsets -8..9
    for (int m = -8; m <= 8; ++m) c[m + 8] += -sx.at(-m);
    for (int j = 0; j <= 1; ++j) {
        const q w = j ? s.alpha : (q)1;
        for (int t = -h; t <= h; ++t) {
            q e = qfact(qo) / (qfact(t + h) * qfact(qo - t - h));
            if ((h - t) % 2) e = -e;
            c[j + t + 8] += xi * w * e;
        }
    }
    // extents
    int reach = 0;
    for (int m = -8; m <= 8; ++m)
        if (s.at(m) != 0) reach = std::max(reach, std::abs(m));
    int cl_lo = 0, cl_hi = 0;
    for (int m = -8; m <= 9; ++m)
        if (c[m + 8] != 0) {
            cl_lo = std::min(cl_lo, m);
            cl_hi = std::max(cl_hi, m);
        }
    const int bh = std::max(reach, std::max(-cl_lo, cl_hi - 1));
    if (bh > kBiasHalf) {
        err = "biased scheme: stencil wider than the supported half-width";
        return CFD_EUNSUPPORTED;
    }
    Scheme r;
    r.kind = 1;
    r.bias = bias;
    r.d = 1;
    r.order = p;
    r.nl = 1;
    r.nc = 1;
    r.m = reach;
    r.mc = std::max(-cl_lo, cl_hi);
    r.bhalf = bh;
    r.balpha = (double)s.alpha;
    for (int m = -kBiasHalf; m <= kBiasHalf; ++m) r.ba[m + kBiasHalf] = (double)s.at(m);
    for (int m = -kBiasHalf; m <= kBiasHalf + 1; ++m) r.bc[m + kBiasHalf] = (double)c[m + 8];
    if (family == 'W') {
        r.emb = M;
        r.ba2 = (double)s.a2;
    }
    if (family == 'U') {   // sampled f'' on every row; the closure row is the mirror's
        r.hermite = 1;
        r.ba2 = (double)s.a2;
        r.bc2 = -(double)s.a2;
    }
    // the left-biased rows as a banded operator, for the generic fields
    r.lhs[kMaxNL - 1] = r.balpha;
    r.lhs[kMaxNL] = 1.0;
    for (int m = -kMaxHalf; m <= kMaxHalf; ++m) r.rhs[kMaxHalf + m] = r.ba[m + kBiasHalf];
    char nm[48];
    std::snprintf(nm, sizeof nm, "(1)%c%d%s", family, M, bias < 0 ? "-" : (bias == 1 ? "+" : (bias == 2 ? "s" : "")));
    r.name = nm;
    out = r;
    return CFD_OK;
}

// Kreiss-Oliger dissipation (Eq. dissdef): Q^(2r) = -(-1)^r / 2^(2r) sigma
// dx^(2r-1) (D_+)^r (D_-)^r.  (D_+ D_-)^r has the centred binomial stencil
// sum_n (-1)^(r-n) C(2r, r+n) f_{k+n} / dx^(2r) (Tab. diss_scheme), so Q^(2r)
// is the explicit symmetric stencil q_n = -(-1)^r sigma 4^-r (-1)^(r-n)
// C(2r, r+n), scaled by dx^-1.  Stored as an explicit scheme of even degree
// 2r (symmetric stencil) with the output scaled by h^-1.
cfd_status design_dissipation(int r, double sigma, Scheme &out, std::string &err) {
    if (r < 1 || r > kMaxHalf) {
        err = "Kreiss-Oliger dissipation: r must be 1..5 (degree 2..10)";
        return CFD_EUNSUPPORTED;
    }
    if (!(sigma >= 0) || !std::isfinite(sigma)) {
        err = "Kreiss-Oliger dissipation: sigma must be finite and >= 0";
        return CFD_EINVAL;
    }
    Scheme s;
    s.d = 2 * r;
    s.hpow = 1;
    s.order = 2;
    s.nl = 0;
    s.m = r;
    s.lhs[kMaxNL] = 1.0;
    const double pre = -((r % 2) ? -1.0 : 1.0) * sigma / std::ldexp(1.0, 2 * r);
    for (int n = -r; n <= r; ++n) {
        double c = 1.0;   // C(2r, r+n)
        for (int i = 1; i <= r + n; ++i) c = c * (2 * r - i + 1) / i;
        const double sg = ((r - n) % 2) ? -1.0 : 1.0;
        s.rhs[kMaxHalf + n] = pre * sg * c;
    }
    char nm[48];
    std::snprintf(nm, sizeof nm, "KO%d[%g]", 2 * r, sigma);
    s.name = nm;
    out = s;
    return CFD_OK;
}

cfd_status scheme_from_name(const std::string &name, Scheme &out, std::string &err) {
    std::string base = name, variant;
    size_t colon = name.find(':');
    if (colon != std::string::npos) {
        base = name.substr(0, colon);
        variant = name.substr(colon + 1);
    }
    if (!(variant.empty() || variant == "E")) {
        err = "unknown closure variant in scheme name '" + name + "'";
        return CFD_EINVAL;
    }
    const bool order_only = (variant == "E");
    // biased: "(1)V3-", "(1)X2+", "(1)X2" (both biases, upwind by a velocity field), "(1)X2s" (the
    // average of both biases)
    if (variant.empty() && base.size() >= 5 && base.compare(0, 3, "(1)") == 0 && (base[3] == 'U' || base[3] == 'V' || base[3] == 'X' || base[3] == 'W') &&
        base[4] >= '1' && base[4] <= '9') {
        const std::string tail = base.substr(5);
        int bias;
        if (tail.empty()) bias = 0;
        else if (tail == "-") bias = -1;
        else if (tail == "+") bias = 1;
        else if (tail == "s") bias = 2;
        else {
            err = "unknown scheme name '" + name + "'";
            return CFD_EINVAL;
        }
        cfd_status bst = design_biased(base[3], base[4] - '0', 0.0, bias, out, err);
        if (bst == CFD_OK) out.name = name;
        return bst;
    }
    if (base.size() < 5 || base[0] != '(' || base[2] != ')' || (base[1] != '1' && base[1] != '2')) {
        err = "unknown scheme name '" + name + "'";
        return CFD_EINVAL;
    }
    const int d = base[1] - '0';
    const std::string kind = base.substr(3);
    cfd_status st;
    if (kind.size() == 4 && kind.compare(0, 3, "P1_") == 0 && kind[3] >= '1' && kind[3] <= '3') {
        int M = kind[3] - '0';
        int order = 2 * M + 2;
        st = design_centred(d, order, 1, M, 0.0, order_only ? order / 2 : order / 2 + 1, !order_only, out, err);
    } else if (kind == "Q1_3[1]" || kind == "Q1_3[4pi/5]") {
        double ec = (kind == "Q1_3[1]") ? 1.0 : 4 * M_PI / 5;
        st = design_centred(d, 6, 1, 3, ec, order_only ? 3 : 4, !order_only, out, err);
    } else if (kind == "QP_O8[1]") {
        st = design_centred(d, 8, 2, 3, 1.0, order_only ? 4 : 5, !order_only, out, err);
    } else if (kind.size() == 2 && kind[0] == 'E' && kind[1] >= '1' && kind[1] <= '5' && !order_only) {
        int M = kind[1] - '0';
        st = design_centred(d, 2 * M, 0, M, 0.0, 0, 0, out, err);
    } else {
        err = "unknown scheme name '" + name + "'";
        return CFD_EINVAL;
    }
    if (st == CFD_OK) out.name = name;
    return st;
}

// The system one iterate of the hybrid closure iteration solves on a block
// line (Eq. iter_center_P): the interior rows of a centred tridiagonal scheme
// on k*_- - c + 1 .. k*_+ + c - 1, with the derivative at k*_- - c and
// k*_+ + c fixed to end values e-, e+.  For c = 2 the extra row k*_- - 1,
//   alpha e- + x_{-1} + alpha x_0 = r_{-1},
// is eliminated into row k*_-:
//   (1 - alpha^2) x_0 + alpha x_1 = r_0 - alpha r_{-1} + alpha^2 e-,
// with r_k the interior stencil at row k, so the system on the block's own
// nodes has an implicit closure row (1 - alpha^2, alpha) whose stencil is
// a_m - alpha a_{m+1} (half-width M + 1) and whose end-value weight is
// gamma = alpha^2; the right end is its mirror image.  For c = 1 the closure
// row is the interior row itself with gamma = -alpha.
cfd_status make_iterated(const Scheme &base, int c, Scheme &out, std::string &err) {
    if (base.nl != 1) {
        err = "the hybrid closure iteration is defined for tridiagonal schemes";
        return CFD_EUNSUPPORTED;
    }
    if (c != 1 && c != 2) {
        err = "iteration end nodes must lie 1 or 2 nodes past the block end";
        return CFD_EINVAL;
    }
    const double al = base.lhs[kMaxNL + 1];
    Scheme s = base;
    s.nc = 1;
    s.ext = 1;
    s.cl_up = al;
    for (int j = 0; j < kMaxNL; ++j)
        for (int m = 0; m <= 2 * kMaxHalf; ++m) s.cl[j][m] = 0.0;
    if (c == 1) {
        s.cl_d0 = 1.0;
        s.gamma = -al;
        s.mc = base.m;
        for (int m = -base.m; m <= base.m; ++m) s.cl[0][kMaxHalf + m] = base.rhs[kMaxHalf + m];
    } else {
        if (base.m + 1 > kMaxHalf) {
            err = "iterated closure stencil wider than the supported half-width";
            return CFD_EUNSUPPORTED;
        }
        s.cl_d0 = 1.0 - al * al;
        s.gamma = al * al;
        s.mc = base.m + 1;
        for (int o = -base.m - 1; o <= base.m; ++o) {
            const double a0 = (o >= -base.m) ? base.rhs[kMaxHalf + o] : 0.0;
            const double a1 = (o + 1 <= base.m) ? base.rhs[kMaxHalf + o + 1] : 0.0;
            s.cl[0][kMaxHalf + o] = a0 - al * a1;
        }
    }
    s.name = base.name + ":iter";
    out = s;
    return CFD_OK;
}

// Taylor check of every row of a scheme (Eq. Tcons): interior rows and the
// explicit closure rows, up to the formal order.
cfd_status check_taylor(const Scheme &s, std::string &err) {
    double scale = 0;
    for (double v : s.rhs) scale = std::fmax(scale, std::fabs(v));
    const double tol = 1e-12 * std::fmax(1.0, scale);
    for (int l = 0; l < s.order + s.d; ++l) {
        long double res = 0;
        for (int k = -kMaxHalf; k <= kMaxHalf; ++k)
            res += (long double)s.rhs[kMaxHalf + k] * std::pow((long double)k, l) / std::tgamma(l + 1.0L);
        if (l >= s.d)
            for (int j = -kMaxNL; j <= kMaxNL; ++j)
                res -= (long double)s.lhs[kMaxNL + j] * std::pow((long double)j, l - s.d) /
                       std::tgamma(l - s.d + 1.0L);
        if (std::fabs((double)res) > tol) {
            char buf[128];
            std::snprintf(buf, sizeof buf, "interior row violates Taylor condition l=%d (residual %.3g)", l,
                          (double)res);
            err = buf;
            return CFD_EINVAL;
        }
        for (int j = 0; j < s.nc; ++j) {
            long double rc = (l == s.d) ? -1.0L : 0.0L;
            for (int k = -kMaxHalf; k <= kMaxHalf; ++k)
                rc += (long double)s.cl[j][kMaxHalf + k] * std::pow((long double)k, l) / std::tgamma(l + 1.0L);
            if (std::fabs((double)rc) > tol) {
                char buf[128];
                std::snprintf(buf, sizeof buf, "closure row %d violates Taylor condition l=%d", j, l);
                err = buf;
                return CFD_EINVAL;
            }
        }
    }
    return CFD_OK;
}

// Centred form the line kernels rely on: they evaluate the interior RHS from
// the m > 0 half of alpha^(0) in symmetric form, so alpha^(0) must be
// antisymmetric for odd d and symmetric for even d, and alpha^(d) symmetric
// (Eq. sch_cent_om uses centred interior rows).  Biased stencils are rejected.
cfd_status check_centred(const Scheme &s, std::string &err) {
    double scale = 0;
    for (double v : s.rhs) scale = std::fmax(scale, std::fabs(v));
    for (double v : s.lhs) scale = std::fmax(scale, std::fabs(v));
    const double tol = 1e-14 * std::fmax(1.0, scale);
    const double sgn = (s.d % 2) ? -1.0 : 1.0;
    for (int k = 1; k <= kMaxHalf; ++k)
        if (std::fabs(s.rhs[kMaxHalf - k] - sgn * s.rhs[kMaxHalf + k]) > tol) {
            err = (s.d % 2) ? "interior stencil alpha^(0) is not antisymmetric (biased stencils are not supported)"
                            : "interior stencil alpha^(0) is not symmetric (biased stencils are not supported)";
            return CFD_EUNSUPPORTED;
        }
    if (s.d % 2 && std::fabs(s.rhs[kMaxHalf]) > tol) {
        err = "interior stencil alpha^(0) of an odd derivative has a nonzero centre weight";
        return CFD_EUNSUPPORTED;
    }
    for (int j = 1; j <= kMaxNL; ++j)
        if (std::fabs(s.lhs[kMaxNL - j] - s.lhs[kMaxNL + j]) > tol) {
            err = "implicit stencil alpha^(d) is not symmetric (biased stencils are not supported)";
            return CFD_EUNSUPPORTED;
        }
    return CFD_OK;
}

// The symbol of the interior rows of D_L, 1 + 2 a1 cos t + 2 a2 cos 2t
// (periodic D of Sec. 2.2; a centred alpha^(d)), must stay positive on
// [0, pi]: a zero makes the periodic matrix singular for some N and the
// closure systems lose the diagonal strength no-pivot elimination relies on.
// With c = cos t it is the quadratic (1 - 2 a2) + 2 a1 c + 4 a2 c^2 on
// [-1, 1]; its minimum is taken at an end or at the vertex.
cfd_status check_symbol(const Scheme &s, std::string &err) {
    const double a1 = s.lhs[kMaxNL + 1], a2 = s.lhs[kMaxNL + 2];
    auto sym = [&](double c) { return (1.0 - 2.0 * a2) + 2.0 * a1 * c + 4.0 * a2 * c * c; };
    double mn = std::fmin(sym(-1.0), sym(1.0));
    if (a2 != 0.0) {
        const double cv = -a1 / (4.0 * a2);
        if (cv > -1.0 && cv < 1.0) mn = std::fmin(mn, sym(cv));
    }
    if (!(mn > 1e-12)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "implicit stencil symbol 1 + 2a1 cos t + 2a2 cos 2t reaches %.3g <= 0 "
                                       "(singular periodic system)", mn);
        err = buf;
        return CFD_ESINGULAR;
    }
    return CFD_OK;
}

int required_ghosts(const Scheme &s, int periodic) {
    if (periodic) return 0;
    if (s.kind == 1) {
        // both biases: left closure row reaches its left half-width, row k*_- + 1
        // the interior left reach - 1, row k*_+ the interior right reach; the
        // right bias mirrors these
        int la = 0, ra = 0, lc = 0;
        for (int m = -kBiasHalf; m <= kBiasHalf; ++m)
            if (s.ba[m + kBiasHalf] != 0) {
                la = std::max(la, -m);
                ra = std::max(ra, m);
            }
        for (int m = -kBiasHalf; m <= kBiasHalf + 1; ++m)
            if (s.bc[m + kBiasHalf] != 0) lc = std::max(lc, -m);
        int need = std::max(lc, std::max(la - 1, ra));
        if (s.emb) need = std::max(need, s.emb + 2);   // the embedded (2)P1_M closure
        return need;
    }
    if (s.nl == 0) return s.m;
    int need = s.m - s.nc;
    for (int j = 0; j < s.nc; ++j) need = std::max(need, s.mc - j);
    return need;
}

}  // namespace cfd
