// Internal declarations of the MI355X compact finite-difference library.
// Shared by the host runtime (cfd_host.cpp, scheme_design.cpp) and the
// device code (cfd_kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cfd.h"

namespace cfd {

constexpr int kMaxNL = 2;        // implicit half-width: tri (1) and penta (2)
constexpr int kMaxHalf = 5;      // RHS / closure stencil half-width
constexpr int kMaxP = 8;         // partitions per line
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kBiasHalf = 5;     // biased schemes: stencil half-width bound

// ---------------------------------------------------------------------------
// Scheme (host only)
// ---------------------------------------------------------------------------
struct Scheme {
    int d = 1;                   // derivative degree
    int order = 0;               // formal order
    int nl = 0;                  // implicit half-width
    int m = 0;                   // interior RHS half-width
    int nc = 0;                  // closure rows per end (= nl)
    int mc = 0;                  // closure half-width
    double lhs[2 * kMaxNL + 1] = {0};         // alpha^(d)_{-2..2}
    double rhs[2 * kMaxHalf + 1] = {0};       // alpha^(0)_{-5..5}
    double cl[kMaxNL][2 * kMaxHalf + 1] = {};  // closure rows k*_- + j, centred at 5
    // Iterated closure (Sec. ssec:domdec_iter): the closure row k*_- is an
    // implicit row of D_L, (cl_d0, cl_up) on columns (k*_-, k*_- + 1), mirrored
    // at k*_+, and its right side also carries gamma times an end value taken
    // from the neighbouring block's previous iterate.
    int ext = 0;
    double cl_d0 = 1.0, cl_up = 0.0, gamma = 0.0;
    // Biased first-degree schemes (Sec. ssec:domdec_drp): kind 1.  Stored as
    // the left-biased scheme, alpha x_{k-1} + x_k = sum_m ba_m f_{k+m}
    // (ba centred at kBiasHalf), and its closure row at k*_-,
    // x_0 + alpha x_1 = sum_m bc_m f_m (bc on -kBiasHalf .. kBiasHalf+1);
    // the right-biased scheme is the mirror image.  bias: -1 left-biased,
    // +1 right-biased, 0 both, combined by the sign of a velocity field.
    // Power of h the output is scaled by (h^-hpow); -1 means d.  Kreiss-Oliger
    // dissipation: stencil of a 2r-th difference (even parity), scaled by h^-1.
    int hpow = -1;
    int kind = 0;
    int bias = -1;
    int bhalf = 0;                 // largest reach of ba / bc (bc may reach bhalf + 1 to the right)
    double balpha = 0.0;
    double ba[2 * kBiasHalf + 1] = {0};
    double bc[2 * kBiasHalf + 2] = {0};
    // W_M: interior rows also carry ba2 dx^2 f''_k, with f'' the centred
    // (2)P1_M (M = emb) solved on the same line with its matched closure;
    // emb = 0 for schemes without an embedded second derivative.
    int emb = 0;
    double ba2 = 0.0;
    // U_M: every row carries a sampled f''_k from an input field (cfd_op
    // aux_field), weight ba2 on interior rows and bc2 on the closure row.
    int hermite = 0;
    double bc2 = 0.0;
    std::string name;
};

// Biased scheme construction (scheme_design.cpp).  family 'U' or 'V' (M = 1..4),
// 'X' or 'W' (M = 1..3; lambda <= 0 takes the value printed with the scheme).
cfd_status design_biased(char family, int M, double lambda, int bias, Scheme &out, std::string &err);
// Kreiss-Oliger dissipation Q^(2r) (Eq. dissdef) as an explicit scheme.
cfd_status design_dissipation(int r, double sigma, Scheme &out, std::string &err);
inline int scale_power(const Scheme &s) { return s.hpow >= 0 ? s.hpow : s.d; }
// A fully determined scheme of the multi-derivative ansatz (Eq. mdAnsatz,
// Eq. Tcons): unknown derivative dr on offsets -L..R (alpha^(dr)_0 = 1),
// sample classes dI[c] on offsets -Lk[c]..Rk[c].  Coefficients in binary128,
// returned as doubles: lhs (L+R+1), then each class's (Lk+Rk+1).
cfd_status taylor_scheme(int dr, int L, int R, int nclass, const int *dI, const int *Lk, const int *Rk,
                         std::vector<double> &coef, int &order, std::string &err);

// Scheme construction (scheme_design.cpp).  Return CFD_OK or an error code
// with the message in `err`.
cfd_status design_centred(int d, int order, int nl, int m, double eta_c, int closure_mc,
                          int matched, Scheme &out, std::string &err);
cfd_status scheme_from_name(const std::string &name, Scheme &out, std::string &err);
cfd_status make_iterated(const Scheme &base, int c, Scheme &out, std::string &err);
cfd_status check_taylor(const Scheme &s, std::string &err);
cfd_status check_centred(const Scheme &s, std::string &err);
cfd_status check_symbol(const Scheme &s, std::string &err);
int required_ghosts(const Scheme &s, int periodic);

// ---------------------------------------------------------------------------
// Device-side plan data (POD, shared with kernels)
// ---------------------------------------------------------------------------

// Table of one operator on one line class (line length N, partition count
// P = N / L, boundary kind), elements of the plan's type:
//   [0, 64)              coefficient block: interior stencil alpha^(0) (11,
//                        centred), left closure rows (2 x 11), right closure
//                        rows (2 x 11, mirror images), alpha^(d) (5)
//   fwd  [p L + i][2]    partition-local LU of D_L, forward factors (l1, l2)
//   bwd  [p L + i][3]    backward factors (u1, u2, 1/d)
//   spk  [p][2nl][L]     spike vectors: local response to the nl left and nl
//                        right neighbour unknowns
//   krow [p][2nl][B]     rows of the inverse of the reduced boundary system,
//                        B = 2 nl P
//   gvec [2][Npad]       iterated closures: response to the left / right end
//                        value (zero otherwise)
constexpr int kCoefA = 0;
constexpr int kCoefCL = 11;
constexpr int kCoefCR = 33;
constexpr int kCoefAlpha = 55;
constexpr int kCoefHdr = 64;

inline int64_t table_elems(int N, int P, int nl) {
    const int64_t L = N / P, B = 2 * nl * P;
    if (nl == 0) return kCoefHdr;
    return kCoefHdr + (int64_t)N * 5 + (int64_t)P * 2 * nl * L + (int64_t)P * 2 * nl * B + 2 * (int64_t)N;
}
inline int64_t table_gvec_offset(int N, int P, int nl) {   // N here is P L
    const int64_t L = N / P, B = 2 * nl * P;
    return kCoefHdr + (int64_t)N * 5 + (int64_t)P * 2 * nl * L + (int64_t)P * 2 * nl * B;
}

// One (block, direction, operator-pass) descriptor, read by every workgroup
// that processes lines of it.  Element offsets/strides.
struct PassDesc {
    int64_t in_base;        // input offset of field 0, interior node (0,0,0)
    int64_t in_fstride;     // input elements per field
    int64_t out_base[2];    // output offset of each op's first field
    int64_t out_fstride;    // output elements per field (= nx ny nz)
    int32_t su, sv, sd;     // input strides along the line's u, v and along the line
    int32_t osu, osv, osd;  // output strides
    int32_t nu, nlines;     // lines: u fastest; nlines = nu * nv
    int32_t N, ng;          // line length, ghost layers
    int32_t periodic;
    int32_t nfield_pass;    // fields this pass covers
    int32_t field0;         // first field index
    int32_t tab[2];         // table index per op
    double hinv[2];         // h^-d per op
    int64_t ev_base[2];     // iterated closures: element offset of each op's end values
                            // (two per line: left, right; field-major), else unused
};

// Biased (upwind) operator on the lines of one block along one direction
// (cfd_biased.hip).  mode: -1 left-biased, +1 right-biased, 0 upwind by the
// sign of the velocity field at vel_base, 2 the mean of both biases.  Coefficient record per table
// (elements of the plan's type): [0] alpha, [1, 12) ba_{-5..5},
// [12, 24) bc_{-5..6}, [24] 1 / (1 - alpha^2), [32, 32 + 65) (-alpha)^n for
// n = 0..64.
constexpr int kBiasRec = 128;
constexpr int kBiasPow = 32;
constexpr int kBiasMaxPN = 64;   // longest line of the partitioned kernel (4 partitions of 16)
struct BiasPass {
    int64_t in_base;        // input offset of field 0, interior node (0,0,0)
    int64_t in_fstride;     // input elements per field
    int64_t vel_base;       // upwind: input offset of the velocity field at interior (0,0,0)
    int64_t out_base;       // output offset of the operator's first field
    int64_t out_fstride;    // output elements per field
    int32_t su, sv, sd;     // input strides (u, v, along the line)
    int32_t osu, osv, osd;  // output strides
    int32_t nu, nlines, N, ng;
    int32_t periodic, mode, tab, hb;
    double hinv;            // 1 / h
    double wrap;            // periodic: 1 / (1 - (-alpha)^N)
    int64_t ev_base;        // iterated closures: first (field 0, line 0) entry of the pass's end values
    // Second-derivative term of W and U schemes: the value for field f at
    // interior node (u, v, k) is src[s2_base + f s2f + u s2u + v s2v + k s2d],
    // src the plan scratch s2 (W: the embedded h^-2 (2)P1_M f, output strides)
    // or, with s2_in, the input (U: the sampled f'' field, input strides, s2f =
    // 0).  Weights in a left-biased row: w2 = ba2 h^2 on interior rows, w2c =
    // bc2 h^2 on the closure row; the right-biased rows take -w2, -w2c.
    // Neither: s2 = null and s2_in = 0.
    const void *s2;
    int64_t s2_base, s2f;
    int32_t s2u, s2v, s2d, s2_in;
    double w2, w2c;
};
// One work item of the partitioned kernel: 64 * (4 / P) lines of one field of
// one pass, P partitions per line (one wave each); of the sweep kernel (lines
// longer than kBiasMaxPN): 64 lines per wave, P = 0.
struct BiasItem {
    int32_t pass, field, line0, P;
};

// One work item: 64 * (waves_for(P) / P) lines of one field of one pass.
// meta: P (partitions per line) in bits 0..3, index of L in the kernel's
// compiled set in bits 4..7, x lines: column chunks C - 1 in bits 8..9.
struct WorkItem {
    int32_t pass;
    int32_t field;
    int32_t line0;
    int32_t meta;
};

// Method-of-lines stage epilogue of the line kernel (extension mode 2).
// Instead of storing its derivative D, an item folds it into one explicit
// Runge-Kutta stage of a state field t:
//   k = (addends) + D,  stage[t] = u0[t] + a k,  acc[t] = acc_in[t] + b k,
// where the addends are derivatives of the same node that other passes of an
// earlier launch stored in the output layout (summed in order).  A pass may
// also update a second field with k = the input value of its own line at the
// node (y and z lines only: the lane holds it in registers).  The state
// arrays have the plan's input layout.  Indexed like the pass descriptors.
struct EpiDesc {
    int64_t add[2];       // output offsets (this block) of the addend derivatives
    int64_t org;          // offset of interior node (0,0,0) within a field
    int32_t mode;         // 0: store the derivative, 1: stage update
    int32_t tgt;          // state field of the stage update
    int32_t self_tgt;     // field updated with k = the line's own value, -1: none
    int32_t nadd;         // addends (0..2)
    int32_t block;        // block index (position in the lattice)
    int32_t dir;          // direction of the pass's lines
    int32_t n[3], ng;     // block extents and ghost layers
    int32_t sy, sz;       // state strides along y and z
};
// Per-launch arguments of the stage epilogue (passed by value to every line
// kernel; read only by the classes compiled with mode 2).  With a lattice
// (lat[0] > 0: the blocks tile a periodic box, block b at (b % bx, b / bx %
// by, b / (bx by))), the state the next stage reads (stage, else acc) also gets
// its face ghosts: a node within ng of a face writes its new value into the
// facing ghost layer of the neighbour across that face.
struct RkArgs {
    const void *u0;
    void *stage;          // nullptr: no stage state
    const void *acc_in;   // may equal u0 (then read once)
    void *acc;
    const EpiDesc *epi;
    const int64_t *in_off;   // input offset of every block (ghost refresh)
    double a, b;
    int32_t lat[3];
    int32_t acc_is_u0;
};

}  // namespace cfd

// ---------------------------------------------------------------------------
// Device entry points (cfd_kernels.hip)
// ---------------------------------------------------------------------------
#include <hip/hip_runtime_api.h>

struct cfd_scheme {
    cfd::Scheme s;
};

namespace cfd {
struct LineClass;

// One pass of a plan: the lines of one block along one direction, for up to
// two operators that share the line data.
struct PassHost {
    int block = 0, dir = 0, field0 = 0, nfield = 1;
    int nops = 1;
    int op[2] = {0, 0};   // plan op indices (output order)
    int sch[2] = {0, 0};  // scheme indices
    int N = 0, ng = 0, periodic = 0, nl = 0, par = 0, mi = 0, hw = 0;
    int ext = 0;          // kernel extension: 1 iterated closures (end-value terms), 2 stage epilogue,
                          // 3 accumulate into the output
    int P = 0, L = 0, lcode = 0;
    int C = 1;            // x lines: column chunks the LDS tile is staged in (divides P)
    const LineClass *cls = nullptr;
    // Passes of the symmetrised mixed derivatives read or write the plan's
    // scratch buffer: iomode 0 input -> output, 1 input -> scratch (first
    // stage), 2 scratch -> scratch, 5 scratch -> output (second stage, after
    // the first), 6 scratch -> output accumulating (third stage, ext 3).  Their
    // strides and offsets are set explicitly (geom) instead of from the block,
    // and hscale multiplies their h^-d.
    // Passes of the fused wave stage: iomode 3 (first launch) and 4 (second
    // launch, after the first), run only by that stage.
    int iomode = 0;
    bool custom = false;
    double hscale = 1.0;
    PassDesc geom{};
};

// Schedule helpers shared by plans and the allocation-free apply (cfd_host.cpp).
size_t exch_bytes(int nl, int nops, int P, bool periodic, size_t es);
size_t x_tile_bytes(int P, int L, int hw, size_t es, int C = 1);
bool chunked(const LineClass *k);
int x_chunks(int P, int L, int hw, size_t es, size_t exch);
int partition_length(const PassHost &ps, bool f32, int P);
int candidate_Ps(const PassHost &ps, bool f32, size_t max_lds, int out[4]);
void fill_pass_desc(PassDesc &q, const cfd_block &b, int64_t in_off, const PassHost &ps, const int64_t out_base[2],
                    const int tab[2], const double hinv[2]);
void place_pass(PassHost &ps, bool f32, int P);
void fill_coef_block(double *cb, const Scheme &s);
cfd_status set_error(cfd_status st, const std::string &msg);   // message for cfd_last_error
size_t pass_lds(const PassHost &ps, bool f32);

// Wavefronts per workgroup of the kernel class that runs items of P
// partitions: 4 for P = 1, 2, 4 (4 / P groups of 64 lines), 8 for P = 8.
inline int waves_for(int P) { return P > 4 ? 8 : 4; }
const LineClass *find_line_class(int f32, int nl, int nops, int par, int mi, int hw, int L, int ext, int wg);
// partition lengths compiled for the class parameters; wg = 0: any workgroup size
int line_class_Ls(int f32, int nl, int nops, int par, int mi, int hw, int *Ls, int cap, int ext = 0, int wg = 0);
hipError_t launch_lines(const void *fn, int wg, int grid, size_t lds, hipStream_t st, const WorkItem *items, int nitems,
                        const int *qoff, const PassDesc *passes, const void *tabs, const int64_t *taboff,
                        const void *in, void *out, const void *ev = nullptr, const RkArgs *rk = nullptr);
hipError_t launch_build_tables(int ntab, const void *specs, double *data, double *scratch, int64_t scratch_per,
                               int *status, hipStream_t st);
hipError_t launch_to_f32(int64_t n, const double *a, float *b, hipStream_t st);
hipError_t launch_xcc_probe(int grid, int *out, hipStream_t st);
hipError_t launch_count_diff(int64_t nwords, const void *a, const void *b, unsigned long long *cnt, hipStream_t st);
hipError_t launch_count_nonfinite(int f32, int64_t n, const void *x, unsigned long long *cnt, hipStream_t st);
size_t tabspec_size();
void fill_tabspec(void *dst, int N, int P, int L, int nl, int nc, int periodic, const double *alpha5,
                  int64_t off, int ext = 0, double cl_d0 = 1.0, double cl_up = 0.0, double gamma = 0.0);
// scratch (doubles) the table builder needs per table
inline int64_t tab_scratch(int P, int L, int nl) {
    const int64_t B = 2 * nl * P, Npad = (int64_t)P * L;
    return 2 * B * B + L + Npad * 5 + B + Npad + 8;
}
}  // namespace cfd

namespace cfd {
hipError_t launch_halo(int f32, void *data, const int64_t *off_dev, int nx, int ny, int nz, int ng, int nfields,
                       int bx, int by, int bz, hipStream_t st);
// pairs_dev: npairs triples (block, face 2 d + side, neighbour); max_face: the most ghost nodes of one face;
// shift 1: vertex-centred blocks (shared extremal nodes)
hipError_t launch_halo_table(int f32, void *data, const int64_t *off_dev, const int *shapes_dev, const int *pairs_dev,
                             int npairs, int nfields, int max_face, int shift, hipStream_t st);
// shared-node averaging along direction d: pairs_dev: npairs (block, + neighbour); max_face: the most nodes of
// one face; ghosted 1: input layout (nslots fields), 0: output layout (nslots operator-fields)
hipError_t launch_shared_avg(int f32, void *data, const int64_t *off_dev, const int *shapes_dev, const int *pairs_dev,
                             int npairs, int nslots, int ghosted, int d, int max_face, hipStream_t st);
hipError_t launch_axpby(int f32, int64_t n, double a, const void *x, double b, void *y, hipStream_t st);
hipError_t launch_xpcy(int f32, int64_t n, const void *x, double c, const void *y, void *z, hipStream_t st);
hipError_t launch_wave_stage(int f32, const void *u0, const void *src, void *stage, const void *acc_in, void *acc,
                             const void *d, const int64_t *in_off, const int64_t *out_off, const int *shapes,
                             const int *unitpre, int nblocks, int nunits, double a, double b, int bx, int by, int bz,
                             hipStream_t st);   // bx = 0: no ghost refresh
}  // namespace cfd

namespace cfd {
// biased (upwind) lines (cfd_biased.hip); hb: stencil half-width class 2..5;
// L: partition length class of the partitioned kernel (8, 12 or 16), 0 for the
// sweep kernel; xdir: lines along x (LDS-staged).
// lds: bytes of dynamic LDS.
bool biased_supported(int hb);
size_t biased_lds(int f32, int hb, int L, int xdir, int P, int N);
// ev: entering end values of an iterated closure (nullptr: the block closure); ends: receives every
// line's end values (nullptr: not written); partitioned kernel only (L > 0)
hipError_t launch_biased(int f32, int hb, int L, int xdir, size_t lds, const BiasItem *items, int nitems,
                         const BiasPass *passes, const void *coefs, const void *in, void *out, const void *ev,
                         void *ends, hipStream_t st);
// recs: npass records (ev base of the pass, of its left neighbour, of its right neighbour, entries)
hipError_t launch_bias_gather(int f32, int npass, int64_t max_entries, const int64_t *recs, const void *ends, void *ev,
                              hipStream_t st);
}  // namespace cfd

namespace cfd {
// hybrid closure iteration (cfd_iterate.hip)
size_t end_weight_spec_size();
size_t iter_op_size();
void fill_end_weight_spec(void *dst, int N, int c, const Scheme &blk, const Scheme &it, int64_t off);
void fill_iter_op(void *dst, int pass, int o, int nbr_m, int nbr_p, int64_t ubase, int nunits, int N, int c, int Npad,
                  int64_t wofs, int64_t gofs, double hinv);
hipError_t launch_end_weights(int ntab, const void *specs, double *data, double *scratch, int stride, hipStream_t st);
hipError_t launch_end_values(int f32, int nops, int max_units, const void *ops, const PassDesc *passes,
                             const double *weights, const void *in, void *ends0, void *endsf, hipStream_t st);
hipError_t launch_iter_ends(int f32, int nops, int max_units, const void *ops, const double *tabs64, const void *endsf,
                            const void *prev, void *next, int gather, hipStream_t st);
}  // namespace cfd

namespace cfd {
hipError_t launch_dense_form(int ntab, const void *tabs, const double *coefs, unsigned char *out, double *scratch,
                             int64_t scratch_per, int *status, hipStream_t st);
const void *dense_apply_fn(int N, bool xdir, bool wide);   // wide: RHS half-width > 3; nullptr: unsupported N
hipError_t launch_dense_apply(const void *fn, int grid, hipStream_t st, const void *items, int nitems,
                              const PassDesc *passes, const void *tabs, const unsigned char *tabdata, const float *in,
                              float *out);
size_t dense_tab_bytes(int N);
size_t dense_tab_struct_size();
size_t dense_item_size();
int dense_item_lines();   // lines per dense work item
void fill_dense_tab(void *dst, int N, int nl, int m, int64_t off);
void fill_dense_item(void *dst, int pass, int field, int line0, int tab);
}  // namespace cfd
