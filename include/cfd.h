/*
 * cfd.h - C ABI of the MI355X compact finite-difference library.
 *
 * The library applies implicit compact finite-difference derivative
 * operators  A f~ = h^-d B f  along the grid lines of 3D mesh blocks held on
 * one GPU (arXiv 2302.14858).  A scheme is the coefficient tuple pair
 * (alpha^(d), alpha^(0)) of the multi-derivative ansatz, Eq. mdAnsatz with
 * d_I = (0), together with the explicit closure stencils used on the rows
 * nearest a block end, Eq. sch_cent_om (Sec. 2.4).  A block has N interior
 * nodes per direction and N_g ghost layers per side (Eq. gridDisc and the
 * figure after it); each direction is either closed by the block closure or
 * periodic (the periodic operator D of Sec. 2.2).
 *
 * Conventions used by every call:
 *  - Return value: cfd_status; CFD_OK on success.  On failure nothing is
 *    enqueued, output handles are left untouched, and cfd_last_error() returns
 *    a thread-local message describing the failure.  No call aborts.
 *  - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensor
 *    storage on the plan's device); every other pointer is host memory.
 *  - Streams are passed as void* holding a hipStream_t (NULL = null stream).
 *    Work is enqueued asynchronously; errors raised by a kernel surface as
 *    CFD_EDEVICE from a later call that synchronises.
 *  - Handles (cfd_scheme*, cfd_plan*) are owned by the library and released
 *    with the matching *_destroy call.  Destroying NULL is a no-op.
 *  - Arrays passed in are copied; the caller keeps ownership.
 */
#ifndef CFD_MI355X_H
#define CFD_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

#define CFD_ABI_VERSION 3

typedef enum {
    CFD_OK = 0,
    CFD_EINVAL = 1,       /* bad argument: null pointer, unknown name, bad layout */
    CFD_EGHOST = 2,       /* ghost width below what the scheme's closure rows reach */
    CFD_ESHAPE = 3,       /* block too short for the closure rows / partitions */
    CFD_ESINGULAR = 4,    /* scheme system singular or not solvable without pivoting */
    CFD_ENOMEM = 5,       /* host or device allocation failed */
    CFD_EDEVICE = 6,      /* HIP runtime error (launch, copy, earlier kernel fault) */
    CFD_EUNSUPPORTED = 7  /* valid request the library does not implement */
} cfd_status;

typedef enum {
    CFD_F64 = 0,          /* FP64 storage and arithmetic */
    CFD_F32 = 1,          /* FP32 storage and arithmetic (tables built in FP64) */
    CFD_MIXED_BF16 = 2    /* FP32 storage; periodic lines only: dense A^-1 B on
                             MFMA in split-BF16 with FP32 accumulation, then one
                             FP64 banded-residual refinement */
} cfd_dtype;

typedef enum {
    CFD_BOUNDARY_CLOSURE = 0,   /* block closure of Eq. sch_cent_om; ghosts are input data */
    CFD_BOUNDARY_PERIODIC = 1   /* the block wraps onto itself; ghosts are not read */
} cfd_boundary;

typedef struct cfd_scheme cfd_scheme;
typedef struct cfd_plan cfd_plan;

/* ------------------------------------------------------------------------ */
/* Library                                                                   */
/* ------------------------------------------------------------------------ */

/* ABI version (CFD_ABI_VERSION of the header the library was built with). */
int cfd_abi_version(void);

/* Thread-local description of the last failure on this thread ("" if none).
 * The string stays valid until the next failing call on the same thread. */
const char *cfd_last_error(void);

/* ------------------------------------------------------------------------ */
/* Schemes (Sec. 2: Eqs. coeffTupDefn, mdAnsatz, Tcons; Sec. 2.4 closures)   */
/* ------------------------------------------------------------------------ */

/* Scheme from the built-in registry, constructed on the host in 113-bit
 * arithmetic from the paper's conditions (Taylor matching, Eq. Tcons;
 * spectral tuning, Eqs. optfunc and gammacut; matched closures, Sec. 2.4).
 * Names:
 *   "(d)P1_M"          d = 1|2, M = 1..3: Pade schemes of Tabs. pade_deg_one/two
 *                      with the matched closures (d)Pbar_{M+2}.
 *   "(d)Q1_3[1]", "(d)Q1_3[4pi/5]"
 *                      tuned tridiagonal schemes of Tabs. num_deg_one/two with
 *                      the matched closures (d)Qbar_4.
 *   "(d)QP_O8[1]"      pentadiagonal (implicit half-width 2), RHS half-width 3,
 *                      formal order 8, tuned with eta_c = 1 by the same
 *                      procedure; matched closures of half-width 5 on the two
 *                      rows nearest each block end.
 *   "(d)EM"            explicit centred schemes of Tab. misc_explicit (M = 1..5),
 *                      e.g. "(1)E3".
 * A suffix ":E" replaces a matched closure by the order-only explicit closure
 * of half-width p (formal order 2p), e.g. "(1)Q1_3[1]:E".
 * Biased first-degree schemes (Sec. ssec:domdec_drp), see
 * cfd_scheme_design_biased:
 *   "(1)VM-", "(1)VM+" M = 1..4: V_M of Tab. ucd_fast, left / right biased,
 *                      with the xi-closure of Tab. ucd_fast_closure.
 *   "(1)XM-", "(1)XM+" M = 1..3: X_M of Tab. ccux_deg_one_col with its closure.
 *   "(1)UM-", "(1)UM+" M = 1..3: U_M of Tab. ucd_slow with the xi-closure of Tab.
 *                      ucd_slow_closure; it samples f'' (cfd_op.aux_field) on
 *                      every row, the closure row included.
 *   "(1)WM-", "(1)WM+" M = 1..3: W_M of Tab. ccuw_deg_one_col (embedded compact
 *                      second derivative) with its closure; "(1)WM" and "(1)WMs"
 *                      as below.
 *   "(1)VM", "(1)XM"   both biases as an upwind pair: an operator with this
 *                      scheme reads a velocity field c (cfd_op.vel_field) and
 *                      returns c d f, left-biased where c > 0 and right-biased
 *                      where c < 0 (Eq. biasderapproxadv).
 *   "(1)VMs", "(1)XMs" the symmetrised scheme: the average of the left- and
 *                      right-biased derivatives (the symmetrisation of biased
 *                      schemes in the decomposition study of Sec. 2.5).
 * out: receives a library-owned handle.  CFD_EINVAL on an unknown name. */
cfd_status cfd_scheme_named(const char *name, cfd_scheme **out);

/* Design a biased first-degree scheme of Sec. ssec:domdec_drp on the host in
 * binary128.  family 'V': V_M (M = 1..4), Eq. defChenSchemes with
 * alpha^(2)_0 = 0, formal order 2M+1, fixed by Taylor matching (Eq. Tcons).
 * family 'X': X_M (M = 1..3), the combination lambda U_M + (1 - lambda)
 * V_{M+1} of Eq. LCslowfast with the f'' sample of U_M replaced by the
 * explicit (2)E_{M+2}, formal order 2M+2; lambda <= 0 takes the value printed
 * with the scheme (Tab. ccux_deg_one_col).  The closure at the block end the
 * bias points away from is the mirror-image scheme plus xi dx^q alpha^(1) .
 * f^(q) over its two implicit nodes, f^(q) from the centred binomial
 * difference (q)E_{q/2} (Tab. diss_scheme), q the first even order above the
 * formal order, xi matching the lowest imaginary term of the interior
 * scheme's wavenumber error (Eqs. ucd_slow_closure_chi, ucd_fast_closure_chi).
 * bias: -1 left-biased (closure row at k*_-, Eq. closure_left_X), +1 right-
 * biased (its mirror image), 0 upwind pair, 2 symmetrised (the mean of both
 * biases; see cfd_scheme_named).
 * Ghost layers needed: the reach of both biases' rows (M + 2 for X_M, M + 1
 * for V_M).  CFD_EUNSUPPORTED outside the ranges above (stencil half-widths
 * above 5), CFD_EINVAL on a bad family or bias. */
cfd_status cfd_scheme_design_biased(char family, int M, double lambda, int bias, cfd_scheme **out);
/* family 'U': U_M (M = 1..3; M = 4 needs a wider closure than the kernels
 * take), Eq. defChenSchemes with the f'' sample, formal order 2M+2; its rows
 * read f'' from an input field (cfd_op.aux_field): interior rows with weight
 * alpha^(2)_0, the closure row with the mirror's, -alpha^(2)_0.
 * family 'W': W_M (M = 1..3, Tab. ccuw_deg_one_col), the same combination
 * keeping alpha^(2)_0 dx^2 f''_k on every interior row, with f'' the compact
 * centred (2)P1_M solved on the same line with its matched explicit closure
 * (lambda <= 0 takes the printed sigma), formal order 2M+2.  At the far end
 * k*_+ (left bias) that f'' is the closure's explicit value, which makes the
 * row there the printed Wtilde; the closure at k*_- (the printed Wbar) is
 * built as above from that explicit row.  In a plan a W operator runs the
 * (2)P1_M pass over the block interior into plan scratch before the biased
 * launches (M + 2 ghost layers; the embedded pass takes the line lengths of the
 * centred second-degree path: closure lines of 3..128 nodes, periodic lines of
 * P partitions of a compiled length, e.g. 8, 12, 16, 24, 32, 48, 64, 96, 128;
 * other lengths give CFD_EUNSUPPORTED at plan creation); cfd_plan_set_iteration
 * refuses plans with W operators. */

/* Kreiss-Oliger dissipation of Eq. dissdef as an operator:
 *   Q^(2r) f = -(-1)^r / 2^(2r) sigma dx^(2r-1) (D_+)^r (D_-)^r f,
 * the explicit centred stencil of (D_+ D_-)^r (the binomial rows of Tab.
 * diss_scheme) times -(-1)^r sigma / 4^r, output scaled by h^-1 (not h^-2r).
 * Used in a plan like any explicit scheme (one direction per operator; the
 * paper adds it in every direction).  Needs r ghost layers on closure lines.
 * r = 1..5 (degree 2..10; Q^(8), r = 4, with sigma = 0.04 is the paper's
 * choice), sigma >= 0.  CFD_EUNSUPPORTED outside that range, CFD_EINVAL for a
 * negative or non-finite sigma. */
cfd_status cfd_scheme_dissipation(int r, double sigma, cfd_scheme **out);

/* Read back a biased scheme: bias (-1, +1, 0), its formal order, alpha =
 * alpha^(1)_{-1} of the left-biased interior row alpha x_{k-1} + x_k =
 * sum_m a_m f_{k+m}, a[11] = a_{-5..5}, and the left closure row
 * x_0 + alpha x_1 = sum_m c_m f_m, c[12] = c_{-5..6}.  Any pointer may be
 * NULL.  CFD_EINVAL for a centred scheme. */
cfd_status cfd_scheme_get_biased(const cfd_scheme *s, int *bias, int *order, double *alpha, double *a11,
                                 double *c12);

/* Read back the second-derivative term of a biased scheme: alpha2 receives
 * alpha^(2)_0 of the left-biased interior row (its right side is
 * sum_m a_m f_{k+m} + alpha2 dx^2 f''_k; the right bias takes -alpha2), m2 the
 * M of the embedded (2)P1_M for W_M (Tab. ccuw_deg_one_col), 0 for U_M (f''
 * sampled from cfd_op.aux_field).  Schemes without the term give 0 and 0.
 * Either pointer may be NULL.  CFD_EINVAL for a centred scheme. */
cfd_status cfd_scheme_get_embedded(const cfd_scheme *s, double *alpha2, int *m2);

/* Fully determined scheme of the multi-derivative ansatz (Eq. mdAnsatz):
 * derivative of degree dr on offsets -L..R (alpha^(dr)_0 = 1) against
 * nclass sample classes, class c of derivative degree dI[c] on offsets
 * -Lk[c]..Rk[c] (e.g. dI = (0, 2) for the Hermite-type schemes, or a biased
 * extent L != R).  As many Taylor conditions (Eq. Tcons) as unknowns are
 * imposed, solved in binary128.  coef receives the L+R+1 left coefficients,
 * then each class's Lk+Rk+1 coefficients, in offset order; cap is its length
 * in doubles (CFD_EINVAL if too small).  order receives the formal order
 * (first violated Taylor condition minus dr).  nclass 1..4, every extent
 * <= 16 nodes.  CFD_ESINGULAR if the conditions are singular. */
cfd_status cfd_taylor_scheme(int dr, int L, int R, int nclass, const int *dI, const int *Lk, const int *Rk,
                             double *coef, int cap, int *order);

/* Design a centred scheme: derivative degree d (1|2), formal order `order`
 * (even), implicit half-width nl (0..2), RHS half-width m (1..5).  When the
 * Taylor conditions leave free coefficients the spectral error of Eq. optfunc
 * with the cut-off weight of Eq. gammacut at eta_c (0 < eta_c <= pi) is
 * minimised.  closure_mc > 0 attaches explicit closures of that half-width on
 * the nl rows nearest each end (matched = 1: lowest error constant matched and
 * the next power removed, Sec. 2.4; matched = 0: Taylor conditions only, which
 * needs closure_mc = order/2).  CFD_EINVAL on inconsistent sizes,
 * CFD_ESINGULAR if the conditions have no solution. */
cfd_status cfd_scheme_design(int d, int order, int nl, int m, double eta_c,
                             int closure_mc, int matched, cfd_scheme **out);

/* Scheme from caller coefficients.
 *   lhs[2nl+1]    alpha^(d)_{-nl..nl}; lhs[nl] must be 1 (normalisation).
 *   rhs[2m+1]     alpha^(0)_{-m..m}.
 *   closure[nc*(2mc+1)]  explicit closure rows for the rows k*_- + j,
 *                 j = 0..nc-1, each alpha^(0)_{-mc..mc}; the right end uses the
 *                 mirror image (-1)^d c[-n].  nc must equal nl (0 for explicit).
 * The Taylor conditions up to `order` are checked on every row (residual
 * <= 1e-12 relative), else CFD_EINVAL.  The interior rows must be centred as in
 * Eq. sch_cent_om: alpha^(d) symmetric and alpha^(0) antisymmetric for odd d,
 * symmetric for even d (to 1e-14 relative), else CFD_EUNSUPPORTED (biased
 * stencils are not implemented).  The symbol of the interior implicit rows,
 * 1 + 2 a1 cos t + 2 a2 cos 2t, must stay positive on [0, pi] (the periodic
 * system of Sec. 2.2 is singular otherwise), else CFD_ESINGULAR.
 * nl <= 2, m <= 5, mc <= 5. */
cfd_status cfd_scheme_create(int d, int order, int nl, const double *lhs, int m,
                             const double *rhs, int nc, int mc, const double *closure,
                             cfd_scheme **out);

/* Read back a scheme.  Any output pointer may be NULL.  Arrays must hold
 * 5 (lhs, centred at index 2), 11 (rhs, centred at 5) and 2*11 (closure rows,
 * each centred at 5) doubles; unused entries are written as 0. */
cfd_status cfd_scheme_get(const cfd_scheme *s, int *d, int *order, int *nl, int *m,
                          int *nc, int *mc, double *lhs5, double *rhs11, double *closure22);

/* Ghost layers the scheme needs for boundary kind b: 0 for periodic; for the
 * closure, the largest reach of any closure or interior row past the block end. */
cfd_status cfd_scheme_required_ghosts(const cfd_scheme *s, cfd_boundary b, int *ng);

void cfd_scheme_destroy(cfd_scheme *s);

/* ------------------------------------------------------------------------ */
/* Plans: a batch of blocks x fields x operators, applied in one step        */
/* ------------------------------------------------------------------------ */

/* One mesh block.  Interior extents n[0..2] = (nx, ny, nz); ng ghost layers on
 * every side; spacing h[0..2]; boundary[0..2] per direction (cfd_boundary).
 * Input layout (elements, from the apply call's input base pointer):
 *   in_offset + f * (nx+2ng)(ny+2ng)(nz+2ng) + ((z+ng)(ny+2ng) + (y+ng))(nx+2ng) + (x+ng)
 *   for field f, interior node (x,y,z); ghosts at negative / >= n coordinates.
 * Output layout (interior only): operator op writes F_op fields (nfields, or
 * 1 when it selects one field), operators packed in order:
 *   out_offset + (S_op + f) * nx*ny*nz + (z*ny + y)*nx + x,  S_op = sum_{o<op} F_o,
 *   f = field index (or 0 for a one-field operator).
 * Offsets of -1 ask the library to pack blocks consecutively in order. */
typedef struct {
    int n[3];
    int ng;
    double h[3];
    int boundary[3];
    long long in_offset;
    long long out_offset;
} cfd_block;

/* One derivative operator: a scheme applied along direction dir (0=x,1=y,2=z)
 * to every field (field = -1) or to one field index.  vel_field: for an
 * upwind pair of biased schemes (e.g. "(1)X2"), the field holding the
 * velocity c; the operator returns c d f with the bias chosen per node by the
 * sign of c (Eq. biasderapproxadv); -1 for every other scheme.
 * dir2: -1, or a second direction != dir: the operator is then the
 * symmetrised mixed derivative 1/2 (D_dir[D_dir2[f]] + D_dir2[D_dir[f]]) of
 * Sec. ssec:z4c with D the first-degree centred scheme `scheme` (block closure
 * or periodic per direction).  On a closed direction i the inner derivative
 * is taken on the lines through the block extended by its ng ghost layers
 * along i (edge ghosts are read), so the outer one has its ghost values.  The
 * plan computes the inner derivatives into a scratch buffer it owns (per
 * block-field and inner direction, the block extended along the outer
 * directions the plan pairs it with; the operators of a plan share them);
 * the first order's outer derivative stores half its value into the output
 * and the second order's adds half of its own.
 * aux_field: for a U_M scheme ("(1)UM-" etc., Tab. ucd_slow), which samples
 * f'' as data, the field holding the second derivative of `field` along dir
 * (read on the interior nodes; field must be a single index); -1 for every
 * other scheme. */
typedef struct {
    const cfd_scheme *scheme;
    int dir;
    int field;
    int vel_field;
    int dir2;
    int aux_field;
} cfd_op;

typedef struct {
    int nblocks;
    const cfd_block *blocks;   /* nblocks entries */
    int nfields;               /* fields per block, >= 1 */
    int nops;                  /* operators, >= 1; output op index = position */
    const cfd_op *ops;
    cfd_dtype dtype;
    int device;                /* HIP device ordinal */
    int flags;                 /* 0 (reserved) */
} cfd_plan_desc;

/* Build a plan: validates every block against every operator (CFD_EGHOST,
 * CFD_ESHAPE), builds and uploads the per-line-class tables (closure and
 * interior coefficients; partition-local LU factors, spike vectors and
 * reduced-system rows, all formed in FP64 on the GPU, Eq. sch_cent_om and its
 * matrix form Eqs. diff_mat_subL/R), the device work lists and the block
 * layout used by the ghost exchange and the stage kernels.  Nothing is
 * allocated later by cfd_apply, cfd_halo_exchange or the stage calls, so
 * they can be captured in a graph.  The first plan on a device also checks
 * how that device deals workgroups to its XCDs (see CFD_SCHED_XCD).
 * Synchronises the device once (table construction). */
cfd_status cfd_plan_create(const cfd_plan_desc *desc, cfd_plan **out);

/* Total input and output sizes in elements for the packed layout (or the
 * extent implied by explicit offsets).  Either pointer may be NULL. */
cfd_status cfd_plan_sizes(const cfd_plan *p, long long *in_elems, long long *out_elems);

/* Resolved per-block offsets (elements).  Arrays of nblocks entries or NULL. */
cfd_status cfd_plan_offsets(const cfd_plan *p, long long *in_offsets, long long *out_offsets);

/* Number of kernel launches one apply enqueues, and the number of work items. */
cfd_status cfd_plan_stats(const cfd_plan *p, int *launches, long long *items);

/* Apply every operator to every field of every block: on every grid line the
 * derivative solves the banded system of Eq. sch_cent_om (block closure) or
 * the circulant system of the periodic D of Sec. 2.2, times h^-d.
 * in_dev: base of the input (element type per dtype), out_dev: base of the
 * output; both 16-byte aligned, else CFD_EINVAL.  Input and output must not
 * overlap.  Enqueued on `stream`; returns immediately.  Allocates nothing. */
cfd_status cfd_apply(cfd_plan *p, const void *in_dev, void *out_dev, void *stream);

/* Capture one apply (the operator of cfd_apply: Eq. sch_cent_om per line)
 * with fixed buffers into a HIP graph owned by the plan (replaces a previous
 * capture).  Buffers as for cfd_apply (16-byte aligned).  Enqueues nothing. */
cfd_status cfd_plan_capture_graph(cfd_plan *p, const void *in_dev, void *out_dev, void *stream);

/* Launch the captured graph (one cfd_apply, Eq. sch_cent_om per line) on
 * `stream`.  CFD_EINVAL if none was captured.  If the runtime could not
 * capture or instantiate the apply, cfd_plan_capture_graph kept its buffers
 * instead and this call enqueues the same apply eagerly (same result; see
 * cfd_plan_graph_status). */
cfd_status cfd_plan_launch_graph(cfd_plan *p, void *stream);

/* How cfd_plan_launch_graph replays: 0 nothing captured, 1 an instantiated
 * HIP graph, 2 the eager fallback (the apply enqueued on each call). */
cfd_status cfd_plan_graph_status(const cfd_plan *p, int *status);

/* Count the non-finite values (NaN, +-inf) in the plan's output extent
 * (cfd_plan_sizes' out_elems elements of out_dev, the plan's element type):
 * a check for results a caller cannot trust (bad input data, an unwritten
 * output).  Enqueued on `stream`, which it synchronises; uses a counter the
 * plan allocated at creation. */
cfd_status cfd_plan_count_nonfinite(cfd_plan *p, const void *out_dev, void *stream, long long *count);

/* Schedule flags. */
#define CFD_SCHED_PERSISTENT 1   /* grid of (occupancy x CUs) workgroups walking the work list */
#define CFD_SCHED_SPLIT_X    2   /* lines along x in a launch of their own */
#define CFD_SCHED_XCD        4   /* block-fields dealt to the 8 XCDs, the same way in
                                    every launch, so the x/y/z passes of a block-field
                                    stay on one L2: a persistent grid walks one queue
                                    per XCD; a per-item grid gets the items in an order
                                    where each workgroup takes the item of its aligned
                                    group of 8 that belongs to the XCD it runs on.  The
                                    per-item form needs the device to deal workgroups
                                    round-robin over 8 XCDs; plan creation checks that
                                    on probe launches and, if it does not hold,
                                    cfd_plan_set_schedule refuses the per-item form
                                    (CFD_EUNSUPPORTED) and the autotuner skips it */
#define CFD_SCHED_CONCURRENT 8   /* the plan's launches (e.g. the x launch and the y/z
                                    launch) run on forked streams at the same time,
                                    joined on the caller's stream before later work;
                                    with CFD_SCHED_SPLIT_X the y/z lines of blocks that
                                    need no LDS for them get a launch of their own; the
                                    biased operators' kernel classes (one launch each)
                                    also run on forked streams */

/* Time the candidate schedules of the operator of cfd_apply (Eq.
 * sch_cent_om per line) on the given buffers and keep the fastest:
 * the launch shape (persistent grid, XCD-aware or not, or one workgroup per
 * item; x lines fused with y/z or split; launches one after another or
 * concurrent), then under that shape the number of partitions per line for
 * every (line length, x or y/z) class, then the launch shape again.  Each
 * candidate's time is the best of three runs of 10 applies.  The winner's
 * output is then compared bit for bit with the plain persistent grid's (same
 * partitions); if they differ the plain shape is kept.  If cache_path
 * is non-NULL the per-class choices are read from / appended to that text
 * file, keyed by device arch, dtype, line length, direction class, band,
 * fused operators and launch shape.  Overwrites out_dev.  Allocates a
 * temporary output-sized buffer for the check.  Synchronises the stream.
 * Invalidates a captured graph.  Biased operators have one launch per kernel
 * class; whether those run one after another or concurrently is tuned last,
 * under the line kernels' schedule (a plan holding only biased operators
 * tunes just that, and reports it as CFD_SCHED_CONCURRENT). */
cfd_status cfd_plan_autotune(cfd_plan *p, const void *in_dev, void *out_dev, void *stream,
                             const char *cache_path);

/* Choose the schedule by hand: lines of length N along x (xlines = 1) or along
 * y/z (xlines = 0) are cut into `partitions` partitions (1, 2, 4, or 8 where a
 * class with 8-wave workgroups is compiled for the band; 0 restores
 * the default); flags is a set of CFD_SCHED_*.  N = 0 only sets the flags.
 * CFD_EINVAL if no compiled kernel fits.  Invalidates a captured graph. */
cfd_status cfd_plan_set_schedule(cfd_plan *p, int N, int xlines, int partitions, int flags);

/* Read back the schedule: persistent receives 0 (one workgroup per item),
 * 1 (persistent grid) or 2 (XCD-aware); split_x the x split
 * flag; for up to cap line classes their (N, xlines, partitions).  n_classes
 * receives the number of classes. */
cfd_status cfd_plan_get_schedule(const cfd_plan *p, int *persistent, int *split_x, int *n_classes, int *N,
                                 int *xlines, int *partitions, int cap);

/* The plan's current schedule flags (a set of CFD_SCHED_*) into *flags. */
cfd_status cfd_plan_get_flags(const cfd_plan *p, int *flags);

void cfd_plan_destroy(cfd_plan *p);

/* Hybrid iteration of the block closures (Sec. ssec:domdec_iter, Eq.
 * iter_center_P; matrix form Eq. iter_scheme).  The plan's blocks tile a
 * periodic box as a bx*by*bz lattice (block index (kz*by + ky)*bx + kx, all
 * blocks the same shape, block closures in every direction, ghosts filled from
 * the neighbours, e.g. by cfd_halo_exchange).  With iterations = n >= 1 every
 * apply returns iterate [n]: iterate 0 is the block closure; iterate i solves
 * the interior tridiagonal rows of each block line on k*_- - 1 .. k*_+ + 1 with
 * the derivative at k*_- - 2 and k*_+ + 2 fixed to the neighbouring blocks'
 * iterate i - 1 at those nodes.  Only tridiagonal centred schemes
 * (CFD_EUNSUPPORTED otherwise); ng must cover the closure and the interior stencil on the row
 * past the block end, max(closure requirement, M + 1) (CFD_EGHOST).
 * iterations = 0 returns to the plain block closure.  Allocates the end-value
 * arrays (two values per line, operator and field, five arrays) and builds the
 * end-node weights in FP64 on the device; invalidates a captured graph.  An
 * apply then enqueues n + 1 small kernels over the end values before the line
 * kernels, and reads the input twice.
 * Biased operators (Eq. iter_left_X and its mirror image) iterate too: for
 * i >= 1 every row of a line takes the interior scheme and the derivative at
 * k*_- - 1 (left bias; k*_+ + 1 right bias), in the ghost layer, is fixed to
 * the neighbouring block's iterate i - 1 there (its last / first node); the
 * upwind pair and the symmetrised mean use the iterated biases.  Each
 * iteration re-runs the biased kernel (one value per line and bias is passed
 * on by a small gather kernel), so an apply costs n + 1 biased passes.  Lines
 * of at most 64 nodes (CFD_EUNSUPPORTED otherwise); ng must cover the closure
 * and the interior stencil on the first and last rows (CFD_EGHOST).
 * Mixed derivatives are not iterated (CFD_EUNSUPPORTED).  CFD_EINVAL if the
 * lattice does not match the plan. */
cfd_status cfd_plan_set_iteration(cfd_plan *p, int iterations, int bx, int by, int bz);

/* ------------------------------------------------------------------------ */
/* Ghost exchange for conforming periodic tilings (the communication step    */
/* of Sec. 2.4, done on the device)                                          */
/* ------------------------------------------------------------------------ */

/* Blocks of one plan that tile a periodic box as a bx*by*bz lattice (block
 * index = (kz*by + ky)*bx + kx, all blocks the same shape) exchange face
 * ghosts: for every field, the ng ghost layers of each face of each block are
 * copied from the facing interior layers of its neighbour.  Edges and corners
 * are not filled (no operator reads them).  data_dev is the plan's input
 * buffer (element type per dtype).  CFD_EINVAL if the lattice does not match
 * the plan's blocks or they differ in shape, CFD_ESHAPE if ng exceeds an
 * extent, CFD_EUNSUPPORTED if one block-field holds 2^31 or more elements or
 * nfields*bx*by*bz exceeds 65535. */
cfd_status cfd_halo_exchange(cfd_plan *p, void *data_dev, int bx, int by, int bz, void *stream);

/* Any conforming tiling (Sec. 2.4: each block's ghost layers are the
 * neighbouring blocks' data): nbr[6 b + f] is the block across face f of
 * block b (f = 0..5 for x-, x+, y-, y+, z-, z+; a block may be its own
 * neighbour, e.g. along a periodic direction), or -1 to leave that face's
 * ghosts as they are (a physical boundary the caller fills).  A face conforms
 * if both blocks have the same extents along the face's two directions and
 * the same ng, and the neighbour has at least ng nodes along the face's
 * normal.  The table is copied to memory the plan allocated at creation (a
 * synchronous copy: call outside graph capture).  Errors: CFD_EINVAL (index
 * out of range), CFD_ESHAPE (a face that does not conform), CFD_EUNSUPPORTED
 * (more than 65535 face x field pairs, or a face of 2^31 or more ghosts). */
cfd_status cfd_plan_set_neighbors(cfd_plan *p, const int *nbr);

/* Face-ghost exchange by the plan's neighbour table: for every field, the ng
 * ghost layers of face f of block b receive the neighbour's ng interior layers
 * facing it (on the + face ghost layer l = the neighbour's interior layer l;
 * on the - face ghost layer l = layer n - ng + l of the neighbour's n nodes),
 * at the same coordinates along the face.  Edges and corners are not filled.
 * data_dev is the plan's input buffer.  One launch, nothing allocated
 * (graph-safe).  CFD_EINVAL if no table has been set. */
cfd_status cfd_halo_exchange_table(cfd_plan *p, void *data_dev, void *stream);

/* Vertex-centred tilings (Eq. gridDisc, G_VC: a block of N_B cells holds
 * N_B + 1 nodes, and neighbours share their extremal node).  As
 * cfd_plan_set_neighbors, but the exchange then continues the ghost layers
 * past the shared node (on the + face ghost layer l = the neighbour's node
 * 1 + l, on the - face node n - 1 - ng + l), the neighbour needs ng + 1
 * nodes along the normal, and every face must be mutual (if block b names q
 * across face f, q names b across the opposite face).  The table also
 * drives cfd_shared_node_average.  Errors as cfd_plan_set_neighbors, and
 * CFD_EINVAL for a face that is not mutual. */
cfd_status cfd_plan_set_neighbors_vc(cfd_plan *p, const int *nbr);

/* Shared-node averaging of vertex-centred blocks (the averaging of shared
 * extremal nodes that the sampling figure and the footnote on the
 * communication matrix of Sec. 2.4 call for): along x, then y, then z, a
 * block's last node and its + neighbour's first node, the same point, both
 * receive the mean of the two values, so a node shared by 2, 4 or 8 blocks
 * ends with the mean of all its copies.  output = 0: data_dev is the plan's
 * input buffer (every field; ghosts untouched); output = 1: the plan's output
 * buffer (every operator and field), e.g. to make the derivatives each block
 * computed at its shared nodes single-valued.  Three launches, nothing
 * allocated.  CFD_EINVAL if no vertex-centred table has been set. */
cfd_status cfd_shared_node_average(cfd_plan *p, void *data_dev, int output, void *stream);

/* ------------------------------------------------------------------------ */
/* Element-wise stage kernels for method-of-lines time stepping (classical   */
/* ERK4, Sec. 3.1): y = a*x + b*y and z = x + c*y over n elements.           */
/* With b = 0, y is overwritten without being read (any prior contents).     */
/* ------------------------------------------------------------------------ */

cfd_status cfd_axpby(cfd_dtype dtype, long long n, double a, const void *x_dev, double b,
                     void *y_dev, void *stream);
cfd_status cfd_xpcy(cfd_dtype dtype, long long n, const void *x_dev, double c, const void *y_dev,
                    void *z_dev, void *stream);

/* One explicit Runge-Kutta stage of the first-order wave system
 *   d_t phi = Pi,  d_t Pi = sum_i d_i psi_i,  d_t psi_i = d_i Pi
 * (the first-order reduction of the wave equation behind the shifted-wave
 * tests of Sec. 3) for a plan with nfields = 5 (phi, Pi, psi_x, psi_y, psi_z)
 * and exactly the six operators [D_x Pi, D_y Pi, D_z Pi, D_x psi_x, D_y psi_y,
 * D_z psi_z] (op = {scheme of degree 1, dir, field}).  src_dev is the stage
 * state and derivs_dev the plan's output computed from it; the right-hand side
 * k is assembled on interior nodes and
 *   stage = u0 + a k      (skipped if stage_dev is NULL; stage may equal src;
 *                          ghosts untouched),
 *   acc   = acc_in + b k  (acc_in NULL means acc itself; acc_in may equal u0,
 *                          which is then read once).
 * u0, src, stage, acc_in and acc are in the plan's input layout (element type
 * per dtype).  Classical RK4 with stage sources u, s, s, s, a = dt/2, dt/2,
 * dt, - and b = dt/6, dt/3, dt/3, dt/6 (s written in place): the first stage
 * takes acc_in = u, the last writes acc = u, so no state copies are needed;
 * then refresh ghosts with cfd_halo_exchange. */
cfd_status cfd_wave_rk_stage(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                             const void *acc_in_dev, void *acc_dev, const void *derivs_dev, double a, double b,
                             void *stream);

/* The same stage for blocks that tile a periodic box as a bx*by*bz lattice
 * (the layout of cfd_halo_exchange), with the ghost exchange fused in: the
 * state the next derivative reads (stage, or acc when stage_dev is NULL) also
 * gets its face ghosts, each interior node within ng of a face writing its new
 * value into the facing ghost layer of the neighbour across that face.  The
 * result equals cfd_wave_rk_stage followed by cfd_halo_exchange on that state,
 * without a second pass over the ghost data.  Errors as cfd_wave_rk_stage, and
 * as cfd_halo_exchange for the lattice. */
cfd_status cfd_wave_rk_stage_halo(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                                  const void *acc_in_dev, void *acc_dev, const void *derivs_dev, double a, double b,
                                  int bx, int by, int bz, void *stream);

/* The same Runge-Kutta stage with the derivatives folded in: the plan's line
 * kernels, instead of storing D_i Pi, update psi_i (and phi, from the Pi they
 * read) in their epilogue, and D_z psi_z updates Pi with D_x psi_x and D_y
 * psi_y, which a first launch stored in work_dev (the plan's output layout and
 * size; only those two operators' slots are written; contents on return are
 * scratch).  Two launches on the stream, in order; nothing is allocated.  The
 * stage arithmetic is that of cfd_wave_rk_stage (k_Pi summed x, y, z in that
 * order), so both give identical results.  bx = by = bz = 0: no ghost refresh;
 * a lattice (bx, by, bz >= 1, as for cfd_wave_rk_stage_halo) also refreshes
 * the face ghosts of the state the next stage reads (stage, or acc when
 * stage_dev is NULL).
 * Buffers: u0, src, stage, acc_in, acc as for cfd_wave_rk_stage, except that
 * stage and acc must not overlap src (the kernels read src while others write
 * the stage state) or each other, and stage must not be u0: run RK4 with two
 * stage buffers in turn (u -> s1 -> s2 -> s1 -> u).  All 16-byte aligned.
 * Errors: CFD_EINVAL (null or aliased buffers, not a wave plan, bad lattice),
 * CFD_EUNSUPPORTED (dense mixed-precision plan, hybrid closure iteration on,
 * or no fused kernel compiled for the scheme's band and line length: the
 * tridiagonal first derivatives with interior half-width up to 3 have one). */
cfd_status cfd_wave_rk_stage_fused(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                                   const void *acc_in_dev, void *acc_dev, void *work_dev, double a, double b, int bx,
                                   int by, int bz, void *stream);

/* ------------------------------------------------------------------------ */
/* Allocation-free apply                                                     */
/* ------------------------------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one
 * operator (scheme s along direction dir) on every line of one block, without
 * a plan and without allocating.  The result equals, bit for bit, that of a
 * plan holding this one operator (cfd_plan_create + cfd_apply with the
 * default schedule).  The solve tables, pass record, work list and the
 * scratch of the FP64 table build that a plan would allocate are kept in one
 * file-scope device array of 8 MiB per GPU, held until the process ends;
 * every step is a kernel launch on `stream`, and nothing is copied from host
 * memory.
 *   blk      the block (in_offset / out_offset are ignored: the input starts
 *            at in_dev, the output at out_dev).
 *   nfields  fields in the input, laid out as for a plan (ghosts included).
 *   field    -1: every field, output [field][z][y][x] (interior only);
 *            k: field k only, output [z][y][x].
 *   dtype    CFD_F64 or CFD_F32 (CFD_MIXED_BF16: CFD_EUNSUPPORTED).
 * Errors as cfd_plan_create for the block and scheme (CFD_EGHOST,
 * CFD_ESHAPE, CFD_EINVAL, 16-byte alignment), and CFD_EUNSUPPORTED when the
 * tables and work list would exceed the 8 MiB array (about half a million
 * work items of 64-256 lines each) or no compiled kernel fits the line
 * length.  A factorisation breakdown (CFD_ESINGULAR at plan creation) is not
 * detected here; schemes are checked for a positive symbol when created.
 * Calls on one GPU share the array, and each call's kernels overwrite it:
 * calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) race and give undefined results.  The first
 * call on a device looks up the array's address (hipGetSymbolAddress); make
 * that call outside graph capture. */
cfd_status cfd_apply_block_noalloc(const cfd_scheme *s, const cfd_block *blk, int dir, int nfields,
                                   int field, cfd_dtype dtype, const void *in_dev, void *out_dev,
                                   void *stream);

/* ------------------------------------------------------------------------ */
/* Test hook                                                                 */
/* ------------------------------------------------------------------------ */

/* Make the library's n-th following device allocation (n = 0: the next one)
 * fail as if the device were out of memory; n < 0 turns the hook off.  For
 * tests of the CFD_ENOMEM paths: every call that allocates returns CFD_ENOMEM
 * and frees what it had allocated.  Process-wide, not thread-safe against
 * concurrent plan creation. */
void cfd_debug_fail_alloc(long long n);

/* Make the next cfd_plan_capture_graph take its eager fallback as if the
 * runtime could not capture (on != 0), for tests of that path. */
void cfd_debug_fail_capture(int on);

#ifdef __cplusplus
}
#endif
#endif /* CFD_MI355X_H */
