// Host-side self test of the library's scheme construction, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU (no GPU code):
// every named scheme, the generators over their parameter ranges, the
// iterated closures and the Taylor / centred / symbol checks, plus invalid
// inputs that must be refused.  Exits non-zero on a failed expectation; the
// sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "cfd_internal.h"

using namespace cfd;

static int g_fail = 0;
#define EXPECT(c)                                                     \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                 \
        }                                                             \
    } while (0)

int main() {
    std::string err;
    const char *names[] = {"(1)P1_1", "(2)P1_1", "(1)P1_2", "(2)P1_2", "(1)P1_3", "(2)P1_3", "(1)Q1_3[1]",
                           "(2)Q1_3[1]", "(1)Q1_3[4pi/5]", "(2)Q1_3[4pi/5]", "(1)QP_O8[1]", "(2)QP_O8[1]",
                           "(1)Q1_3[1]:E", "(2)QP_O8[1]:E", "(1)E1", "(1)E3", "(2)E4", "(1)E5", "(1)V1-", "(1)V4+",
                           "(1)X1", "(1)X2-", "(1)X3+"};
    for (const char *n : names) {
        Scheme s;
        cfd_status st = scheme_from_name(n, s, err);
        EXPECT(st == CFD_OK);
        if (st != CFD_OK) std::printf("  %s: %s\n", n, err.c_str());
        if (s.kind == 0) {
            EXPECT(check_taylor(s, err) == CFD_OK);
            EXPECT(check_centred(s, err) == CFD_OK);
            if (s.nl > 0) EXPECT(check_symbol(s, err) == CFD_OK);
            if (s.nl == 1) {
                Scheme it;
                EXPECT(make_iterated(s, 2, it, err) == CFD_OK);
                EXPECT(make_iterated(s, 1, it, err) == CFD_OK);
                EXPECT(make_iterated(s, 3, it, err) == CFD_EINVAL);
            }
        }
        EXPECT(required_ghosts(s, 0) >= 1);
        EXPECT(required_ghosts(s, 1) == 0);
    }
    const char *bad_names[] = {"", "(", "(3)P1_1", "(1)P1_9", "(1)Q1_3[2]", "(1)X4", "(1)V0", "(1)X2*", "(2)X2",
                               "(1)Q1_3[1]:F", "(1)E9", "KO8", "(1)E3:E"};
    for (const char *n : bad_names) {
        Scheme s;
        EXPECT(scheme_from_name(n, s, err) != CFD_OK);
    }
    // centred generator over its range
    for (int d = 1; d <= 2; ++d)
        for (int nl = 0; nl <= 2; ++nl)
            for (int m = 1; m <= 5; ++m)
                for (int order = 2; order <= 10; order += 2) {
                    Scheme s;
                    const int mc = (nl > 0) ? order / 2 + 1 : 0;
                    cfd_status st = design_centred(d, order, nl, m, 1.0, mc <= 5 ? mc : 0, 1, s, err);
                    EXPECT(st == CFD_OK || st == CFD_EINVAL || st == CFD_ESINGULAR);
                }
    {
        Scheme s;
        EXPECT(design_centred(3, 6, 1, 3, 1.0, 4, 1, s, err) == CFD_EINVAL);
        EXPECT(design_centred(1, 6, 3, 3, 1.0, 4, 1, s, err) == CFD_EINVAL);
        EXPECT(design_centred(1, 6, 1, 6, 1.0, 4, 1, s, err) == CFD_EINVAL);
        EXPECT(design_centred(1, 6, 1, 3, -1.0, 4, 1, s, err) == CFD_EINVAL);
    }
    // biased generator
    for (char fam : {'U', 'V', 'X', 'W'})
        for (int M = 0; M <= 6; ++M)
            for (int bias = -2; bias <= 3; ++bias) {
                Scheme s;
                cfd_status st = design_biased(fam, M, 0.0, bias, s, err);
                // U_4 designs but its closure is wider than the compiled half-width
                const bool ok_range = (fam == 'V') ? (M >= 1 && M <= 4) : (M >= 1 && M <= 3);
                if (bias < -1 || bias > 2) EXPECT(st == CFD_EINVAL);
                else if (ok_range) EXPECT(st == CFD_OK);
                else EXPECT(st == CFD_EUNSUPPORTED);
            }
    {
        Scheme s;
        EXPECT(design_biased('Q', 2, 0.0, 0, s, err) == CFD_EINVAL);
        EXPECT(design_biased('X', 2, 0.5, -1, s, err) == CFD_OK);
        EXPECT(design_biased('W', 2, 0.5, 1, s, err) == CFD_OK && s.emb == 2 && s.ba2 != 0.0);
        EXPECT(design_biased('U', 3, 0.0, 0, s, err) == CFD_OK && s.hermite == 1 && s.bc2 == -s.ba2);
        EXPECT(required_ghosts(s, 0) == 5 && required_ghosts(s, 1) == 0);
    }
    // dissipation
    for (int r = 0; r <= 6; ++r) {
        Scheme s;
        cfd_status st = design_dissipation(r, 0.04, s, err);
        EXPECT((r >= 1 && r <= 5) ? st == CFD_OK : st == CFD_EUNSUPPORTED);
    }
    {
        Scheme s;
        EXPECT(design_dissipation(4, -1.0, s, err) == CFD_EINVAL);
        EXPECT(design_dissipation(4, NAN, s, err) == CFD_EINVAL);
    }
    // general Taylor solver
    {
        std::vector<double> c;
        int order = 0;
        const int dI1[1] = {0}, L1[1] = {2}, R1[1] = {2};
        EXPECT(taylor_scheme(1, 1, 1, 1, dI1, L1, R1, c, order, err) == CFD_OK && order == 6 && c.size() == 8);
        const int dI2[2] = {0, 2}, L2[2] = {1, 0}, R2[2] = {2, 0};
        EXPECT(taylor_scheme(1, 0, 1, 2, dI2, L2, R2, c, order, err) == CFD_OK && order == 5);
        const int big[1] = {9};
        EXPECT(taylor_scheme(1, 9, 9, 1, dI1, big, big, c, order, err) == CFD_EINVAL);
        EXPECT(taylor_scheme(1, 1, 1, 0, dI1, L1, R1, c, order, err) == CFD_EINVAL);
        EXPECT(taylor_scheme(1, 1, 1, 1, nullptr, L1, R1, c, order, err) == CFD_EINVAL);
    }
    // caller coefficients: biased and non-positive-symbol stencils are refused
    {
        Scheme s;
        s.d = 1;
        s.order = 2;
        s.nl = 1;
        s.m = 1;
        s.lhs[kMaxNL] = 1.0;
        s.rhs[kMaxHalf - 1] = -1.0;
        s.rhs[kMaxHalf] = 1.0;
        EXPECT(check_centred(s, err) == CFD_EUNSUPPORTED);
        s.rhs[kMaxHalf - 1] = -0.5;
        s.rhs[kMaxHalf] = 0.0;
        s.rhs[kMaxHalf + 1] = 0.5;
        EXPECT(check_centred(s, err) == CFD_OK);
        s.lhs[kMaxNL - 1] = s.lhs[kMaxNL + 1] = 0.5;   // symbol 1 + cos t reaches 0
        EXPECT(check_symbol(s, err) == CFD_ESINGULAR);
    }
    std::printf("%s (%d failures)\n", g_fail ? "FAIL" : "OK", g_fail);
    return g_fail ? 1 : 0;
}
