// Host runtime and C ABI of the MI355X compact finite-difference library.
//
// A plan turns (blocks x fields x operators) into:
//  * passes: one per (block, direction, field selection, fused operator
//    group); a pass sweeps every line of that direction once and evaluates up
//    to two operators that share the line data (e.g. the first and second
//    derivative of the same field);
//  * tables: per (operator scheme, line length, partition count, boundary)
//    the coefficient block plus the FP64 solve tables built on the GPU;
//  * work items of 64 lines, grouped into launch groups by compiled kernel
//    variant and partition count.  One apply = one kernel launch per group,
//    each a persistent grid over its items (or one workgroup per item).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "cfd_internal.h"
#include "cfd_kernels_reg.h"

using namespace cfd;

namespace {

thread_local std::string g_err;

cfd_status fail(cfd_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

cfd_status hip_fail(hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? CFD_ENOMEM : CFD_EDEVICE, m);
}

// Every device allocation of the library goes through dmalloc.  A test hook
// (cfd_debug_fail_alloc) can make the n-th following allocation fail as if the
// device were out of memory, to check that every failure path returns
// CFD_ENOMEM and frees what it had allocated.
std::atomic<long long> g_alloc_fail_after{-1};
std::atomic<bool> g_fail_capture{false};   // test hook: the next capture falls back to eager replay

hipError_t dmalloc(void **ptr, size_t bytes) {
    long long n = g_alloc_fail_after.load();
    while (n >= 0) {
        if (g_alloc_fail_after.compare_exchange_weak(n, n - 1)) {
            if (n == 0) {
                *ptr = nullptr;
                return hipErrorOutOfMemory;
            }
            break;
        }
    }
    return hipMalloc(ptr, bytes);
}

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace

namespace {

struct Group {
    const void *fn;
    size_t lds;
    int64_t item0, nitems;
    int grid_persist;
    int qoff_index = -1;   // offset of this group's 9 queue bounds in d_qoff (XCD-aware mode)
    int iomode = 0;        // buffers: 0 input -> output, 1 input -> scratch, 2 scratch -> scratch,
                           // 5 scratch -> output, 6 the same accumulating;
                           // 3 and 4: the two launches of the fused wave stage
    int wg = 4;            // wavefronts per workgroup of the kernel class
};

struct TabKey {
    int sch, N, P, L, periodic;
    bool operator<(const TabKey &o) const {
        return std::tie(sch, N, P, L, periodic) < std::tie(o.sch, o.N, o.P, o.L, o.periodic);
    }
};

}  // namespace

struct cfd_plan {
    int device = 0;
    cfd_dtype dtype = CFD_F64;
    int nfields = 1;
    std::vector<cfd_block> blocks;
    std::vector<Scheme> schemes;          // one per op, then the second derivatives W operators embed
    std::vector<cfd_op> ops;              // scheme pointers not used after creation
    std::vector<int> op_nf;               // fields each op writes
    std::vector<int64_t> op_slot;         // S_op
    std::vector<int64_t> in_off, out_off;
    int64_t in_elems = 0, out_elems = 0;
    std::vector<PassHost> passes;
    std::map<std::pair<int, int>, int> sched_P;   // (N, x-direction) -> partitions per line
    bool persistent = true;
    bool split_x = false;                 // x-lines in a launch of their own
    bool xcd = false;                     // XCD-aware queues (persistent grid only)
    bool concurrent = false;              // kernel groups on forked streams, joined at the end
    bool bconcurrent = false;             // the biased kernel classes on forked streams
    int cus = 256;
    size_t max_lds = 65536;
    bool xcd_interleave_ok = false;       // dispatch check passed: the XCD-interleaved per-item order covers every item
    // hybrid closure iteration: iterations (0: off), end-node offset c, lattice
    int iter_n = 0, iter_c = 2, lat[3] = {0, 0, 0};
    std::vector<Scheme> base_schemes;     // the block-closure schemes while schemes holds the iterated ones
    DevBuf d_iops, d_weights, d_ends0, d_endsf, d_ebufA, d_ebufB, d_ev;
    int n_iops = 0, iter_max_units = 0;
    int64_t nunits = 0;                   // 64-node interior pieces of all blocks (stage kernels)
    // device state rebuilt by build()
    DevBuf d_tab64, d_tab32, d_taboff, d_pass, d_items, d_inoff, d_qoff, d_outoff, d_shapes;
    DevBuf d_dense, d_dense_specs;        // dense mixed-precision tables
    // biased (upwind) operators: one pass per (block, op), work items grouped
    // by stencil half-width class, coefficient records per op
    struct BGroup {
        int hb = 0, L = 0, xdir = 0;   // L = 0: sweep kernel
        size_t lds = 0;
        int64_t item0 = 0, nitems = 0;
    };
    std::vector<BGroup> bgroups;
    int64_t nbitems = 0;
    DevBuf d_bpass, d_bitems, d_bcoef;
    // iterated biased closures: per biased pass its block, operator and end
    // entries (fields x lines); end values (entering, and written by each
    // iterate) and the gather records, built by cfd_plan_set_iteration
    std::vector<std::array<int64_t, 4>> bpinfo;   // block, op, ev_base, entries
    int64_t bev_entries = 0, bev_max = 0;
    DevBuf d_bev, d_bends, d_bgrecs;
    // scratch of the mixed derivatives' first stage and of the W operators'
    // embedded second derivative (elements)
    int64_t mscr_elems = 0;
    DevBuf d_mscr;
    int64_t n_mixed = 0;                  // (block, mixed-derivative operator) pairs
    // W operators: scheme index of the embedded (2)P1_M per op (-1: none), and
    // per (block, op) the scratch offset of its first field's h^-2 (2)P1_M f,
    // written by line passes that run before the biased launches
    std::vector<int> emb_sch;
    std::map<std::pair<int, int>, int64_t> emb_off;
    std::vector<Group> groups;
    int64_t nitems = 0;
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> aux;         // one per group beyond the first (concurrent mode)
    std::vector<hipEvent_t> ev;           // fork event, then one join event per aux stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *eager_in = nullptr;       // capture fallback: the buffers replayed eagerly
    void *eager_out = nullptr;
    DevBuf d_count;                       // counter of cfd_plan_count_nonfinite
    // fused wave stage: the wave operators once more as passes of iomode 3 / 4
    // with stage epilogues (EpiDesc per pass); ok once their kernels exist
    bool wave_fused = false, wave_fused_ok = false;
    DevBuf d_epi;
    // ghost exchange by neighbour table: (block, face, neighbour) triples,
    // room for every face allocated at creation; n_hpairs < 0 until set
    DevBuf d_hpairs;
    int n_hpairs = -1, hface_max = 0;
    // vertex-centred tables: ghosts continue past the shared node (hshift 1);
    // (block, + neighbour) pairs per direction for the shared-node average
    int hshift = 0;
    DevBuf d_vpairs;
    int nvp[3] = {0, 0, 0}, voff[3] = {0, 0, 0}, vface_max[3] = {0, 0, 0};

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        eager_in = nullptr;
        eager_out = nullptr;
    }
    // kept across rebuilds of the launch groups (autotuning, schedules)
    void release_biased_iteration() {
        d_bev.release();
        d_bends.release();
        d_bgrecs.release();
        bev_max = 0;
    }
    void release_iteration() {
        d_iops.release();
        d_weights.release();
        d_ends0.release();
        d_endsf.release();
        d_ebufA.release();
        d_ebufB.release();
        d_ev.release();
        n_iops = 0;
        iter_max_units = 0;
    }
    void release() {
        drop_graph();
        d_tab64.release();
        d_tab32.release();
        d_taboff.release();
        d_pass.release();
        d_items.release();
        d_inoff.release();
        d_qoff.release();
        d_outoff.release();
        d_shapes.release();
        d_dense.release();
        d_dense_specs.release();
        d_bpass.release();
        d_bitems.release();
        d_bcoef.release();
        d_mscr.release();
        d_count.release();
        d_epi.release();
        d_hpairs.release();
        release_biased_iteration();
        d_vpairs.release();
        release_iteration();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
        for (hipStream_t a : aux) (void)hipStreamDestroy(a);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        aux.clear();
        ev.clear();
    }
};

namespace cfd {

// Exchange-area bytes an item needs: partition coupling (P > 1) or the
// periodic wrap; none for a single-partition closure line.  Same layout as
// the kernel's (waves_for(P) / P line groups x operators x 64 lanes x
// (2 nl P | 1)).
size_t exch_bytes(int nl, int nops, int P, bool periodic, size_t es) {
    if (nl <= 0 || (P <= 1 && !periodic)) return 0;
    return (size_t)(waves_for(P) / P) * nops * kWave * (size_t)((2 * nl * P) | 1) * es;
}

// Tile bytes an x item with P partitions of L rows needs in LDS: 64
// (waves_for(P) / P) lines by the columns of one chunk (P/C partitions plus
// the halo).
size_t x_tile_bytes(int P, int L, int hw, size_t es, int C) {
    return (size_t)(kWave * waves_for(P) / P) * (size_t)((P / C * L + 2 * hw) | 1) * es;
}

// Column chunks for x lines: the fewest (dividing P) that keep tile and
// exchange area within 80 KiB, so two workgroups share a CU (the line
// classes' registers allow no more than that for long partitions); long lines
// are then staged chunk by chunk.
// Only kernel classes compiled with the chunk loop (partitions of 48 rows or
// more) stage in chunks.
bool chunked(const LineClass *k) {
    int m = 0;
    for (int j = 0; j < k->nL; ++j) m = std::max(m, k->Ls[j]);
    return m >= 48;
}

int x_chunks(int P, int L, int hw, size_t es, size_t exch) {
    for (int C = 1; C <= P; C *= 2)
        if (std::max(x_tile_bytes(P, L, hw, es, C), exch) <= 81920) return C;
    return P;
}

// Partition length for P partitions of an N-node line: the smallest compiled
// L with P L >= N (P L == N for periodic lines) whose last partition holds
// every right-closure row.  0 if none.  For a closure line the ring of an
// inner partition, HW nodes past its last row with HW the half-width the
// kernel class is compiled for, must stay inside the stored line (N + ng
// nodes): the kernel loads it without bounds checks.
int partition_length(const PassHost &ps, bool f32, int P) {
    int Ls[16];
    const int n = line_class_Ls(f32, ps.nl, ps.nops, ps.par, ps.mi, ps.hw, Ls, 16, ps.ext, waves_for(P));
    int best = 0;
    for (int i = 0; i < n; ++i) {
        const int L = Ls[i];
        if ((int64_t)P * L < ps.N) continue;
        if (ps.periodic && P * L != ps.N) continue;
        if (ps.nl > 0 && L < 2 * ps.nl) continue;
        if ((P - 1) * L > ps.N - ps.nl) continue;   // every right-closure row in the last partition
        if (P > 1 && (P - 1) * L >= ps.N) continue;                            // no empty partition
        if (!ps.periodic && P > 1 && ps.dir != 0) {
            const LineClass *k = find_line_class(f32, ps.nl, ps.nops, ps.par, ps.mi, ps.hw, L, ps.ext, waves_for(P));
            if (!k || (P - 1) * L + k->hw > ps.N + ps.ng) continue;
        }
        if (!best || L < best) best = L;
    }
    return best;
}

// Candidate partition counts for a pass, best first, into out[0..3); returns
// how many.  A candidate needs a compiled class with a fitting L, and (x
// lines) an LDS tile that fits next to the exchange area.  No heap use (the
// allocation-free apply calls this too).
int candidate_Ps(const PassHost &ps, bool f32, size_t max_lds, int out[4]) {
    int ok[4], Lok[4], n = 0;
    const size_t es = f32 ? 4 : 8;
    for (int P = 1; P <= 8; P *= 2) {
        const int L = partition_length(ps, f32, P);
        if (!L) continue;
        const LineClass *k = find_line_class(f32, ps.nl, ps.nops, ps.par, ps.mi, ps.hw, L, ps.ext, waves_for(P));
        if (!k) continue;
        if (ps.periodic && k->hw > ps.N) continue;
        size_t lds = exch_bytes(ps.nl, ps.nops, P, ps.periodic, es);
        if (ps.dir == 0)   // the x tile and the exchange area share the LDS
            lds = std::max(lds, x_tile_bytes(P, L, k->hw, es, chunked(k) ? x_chunks(P, L, k->hw, es, lds) : 1));
        if (lds > max_lds) continue;
        ok[n] = P;
        Lok[n] = L;
        ++n;
    }
    // default preference: y/z lines: fewest partitions with L <= 24 (register
    // budget); x lines: L <= 16 (LDS tile); then the rest, most partitions first
    const int Lcap = ps.dir == 0 ? 16 : 24;
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (Lok[i] <= Lcap) out[m++] = ok[i];
    for (int i = n - 1; i >= 0; --i)
        if (Lok[i] > Lcap) out[m++] = ok[i];
    return m;
}

std::vector<int> candidate_Ps(const PassHost &ps, bool f32, size_t max_lds) {
    int c[4];
    const int n = candidate_Ps(ps, f32, max_lds, c);
    return std::vector<int>(c, c + n);
}

// Strides, offsets and line counts of one pass over block b along ps.dir.
// in_off: the block's input offset; out_base[o]: where operator o's first
// field starts in the output; tab[o]: table index; hinv[o] = h^-d.
void fill_pass_desc(PassDesc &q, const cfd_block &b, int64_t in_off, const PassHost &ps, const int64_t out_base[2],
                    const int tab[2], const double hinv[2]) {
    const int64_t ng = b.ng;
    const int64_t PX = b.n[0] + 2 * ng, PY = b.n[1] + 2 * ng, PZ = b.n[2] + 2 * ng;
    const int64_t s_in[3] = {1, PX, PX * PY};
    const int64_t s_out[3] = {1, b.n[0], (int64_t)b.n[0] * b.n[1]};
    const int d = ps.dir;
    const int u = (d == 0) ? 1 : 0;
    const int v = (d == 2) ? 1 : 2;
    std::memset(&q, 0, sizeof q);
    q.in_base = in_off + ng * (s_in[0] + s_in[1] + s_in[2]);
    q.in_fstride = PX * PY * PZ;
    for (int o = 0; o < ps.nops; ++o) {
        q.out_base[o] = out_base[o];
        q.tab[o] = tab[o];
        q.hinv[o] = hinv[o];
    }
    q.out_fstride = (int64_t)b.n[0] * b.n[1] * b.n[2];
    q.su = (int32_t)s_in[u];
    q.sv = (int32_t)s_in[v];
    q.sd = (int32_t)s_in[d];
    q.osu = (int32_t)s_out[u];
    q.osv = (int32_t)s_out[v];
    q.osd = (int32_t)s_out[d];
    q.nu = b.n[u];
    q.nlines = b.n[u] * b.n[v];
    q.N = ps.N;
    q.ng = b.ng;
    q.periodic = ps.periodic;
    q.nfield_pass = ps.nfield;
    q.field0 = ps.field0;
}

cfd_status set_error(cfd_status st, const std::string &msg) { return fail(st, msg); }

// Coefficient block of a table (the first kCoefHdr elements): interior
// stencil, left closure rows, right closure rows (mirror images,
// (-1)^d c[-m]) and alpha^(d).
void fill_coef_block(double *cb, const Scheme &s) {
    for (int i = 0; i < kCoefHdr; ++i) cb[i] = 0.0;
    for (int m = 0; m < 11; ++m) cb[kCoefA + m] = s.rhs[m];
    const double sgn = (s.d % 2) ? -1.0 : 1.0;
    for (int j = 0; j < kMaxNL; ++j)
        for (int m = -kMaxHalf; m <= kMaxHalf; ++m) {
            cb[kCoefCL + j * 11 + 5 + m] = s.cl[j][5 + m];
            cb[kCoefCR + j * 11 + 5 + m] = sgn * s.cl[j][5 - m];
        }
    for (int j = 0; j < 5; ++j) cb[kCoefAlpha + j] = s.lhs[j];
}

// Kernel class, partition length and LDS bytes of a pass with P partitions.
void place_pass(PassHost &ps, bool f32, int P) {
    ps.P = P;
    ps.L = partition_length(ps, f32, P);
    ps.cls = find_line_class(f32, ps.nl, ps.nops, ps.par, ps.mi, ps.hw, ps.L, ps.ext, waves_for(P));
    ps.lcode = 0;
    for (int j = 0; j < ps.cls->nL; ++j)
        if (ps.cls->Ls[j] == ps.L) ps.lcode = j;
    const size_t es = f32 ? 4 : 8;
    ps.C = (ps.dir == 0 && chunked(ps.cls))
               ? x_chunks(ps.P, ps.L, ps.cls->hw, es, exch_bytes(ps.nl, ps.nops, ps.P, ps.periodic, es))
               : 1;
}

size_t pass_lds(const PassHost &ps, bool f32) {
    const size_t es = f32 ? 4 : 8;
    size_t lds = exch_bytes(ps.nl, ps.nops, ps.P, ps.periodic, es);
    if (ps.dir == 0) lds = std::max(lds, x_tile_bytes(ps.P, ps.L, ps.cls->hw, es, ps.C));   // shared area
    return lds;
}

}  // namespace cfd

namespace {

size_t elem_size(cfd_dtype t) { return t == CFD_F64 ? 8 : 4; }   // F32 and MIXED_BF16 store FP32

constexpr int kXCDq = 8;   // queues of the XCD-aware schedule (one per XCD)

// Passes that only the fused wave stage runs (iomode 3 and 4).
inline bool fused_iomode(int m) { return m == 3 || m == 4; }
inline bool fused_pass(const PassHost &ps) { return fused_iomode(ps.iomode); }
// Launch stage of a group of the plain apply: 0 reads the input, 1 reads what
// stage 0 left in the scratch, 2 accumulates into what stage 1 stored.
inline int apply_stage(int m) { return (m == 0 || m == 1) ? 0 : (m == 6 ? 2 : 1); }

// The wave system's operators in the order the stage kernels expect:
// D_x Pi, D_y Pi, D_z Pi, D_x psi_x, D_y psi_y, D_z psi_z (first degree).
bool is_wave_plan(const cfd_plan *p) {
    static const int want[6][2] = {{0, 1}, {1, 1}, {2, 1}, {0, 2}, {1, 3}, {2, 4}};
    if (p->nfields != 5 || p->ops.size() != 6) return false;
    for (int o = 0; o < 6; ++o)
        if (p->ops[o].dir != want[o][0] || p->ops[o].field != want[o][1] || p->schemes[o].d != 1 ||
            p->schemes[o].kind != 0 || p->ops[o].dir2 >= 0)
            return false;
    return true;
}

// Pass descriptors (strides, offsets, h^-d) of every pass; table indices from pass_tab.
std::vector<PassDesc> pass_descs(const cfd_plan *p, const std::vector<std::array<int, 2>> &pass_tab) {
    std::vector<PassDesc> pd(p->passes.size());
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const PassHost &ps = p->passes[i];
        const cfd_block &b = p->blocks[ps.block];
        const int64_t npts = (int64_t)b.n[0] * b.n[1] * b.n[2];
        int64_t ob[2] = {0, 0};
        int tab[2] = {0, 0};
        double hinv[2] = {0, 0};
        for (int o = 0; o < ps.nops; ++o) {
            ob[o] = p->out_off[ps.block] + p->op_slot[ps.op[o]] * npts;
            tab[o] = pass_tab[i][o];
            hinv[o] = ps.hscale / std::pow(b.h[ps.dir], scale_power(p->schemes[ps.sch[o]]));
        }
        if (ps.custom) {
            pd[i] = ps.geom;
            pd[i].tab[0] = tab[0];
            pd[i].hinv[0] = hinv[0];
        } else {
            fill_pass_desc(pd[i], b, p->in_off[ps.block], ps, ob, tab, hinv);
        }
    }
    return pd;
}

cfd_status build_dense(cfd_plan *p);

// Does this device deal a launch's workgroups round-robin over its kXCDq
// XCDs, so that every aligned group of kXCDq consecutive workgroups runs on
// kXCDq distinct XCDs?  The XCD-interleaved per-item order (each workgroup
// takes the item of its group that belongs to the XCD it runs on) covers every
// item only then.  Checked once per device on probe launches of several grid
// sizes (the first XCD of a launch varies), the result cached.
bool xcd_dispatch_ok(int device) {
    static std::mutex mu;
    static std::map<int, bool> known;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(device);
    if (it != known.end()) return it->second;
    bool ok = true;
    const int grids[] = {8 * 512, 8 * 64 + 3, 8 * 300 + 5, 8 * 1024, 8 * 33 + 1, 8 * 700};
    int *d = nullptr;
    std::vector<int> h(8 * 1024);
    if (dmalloc((void **)&d, h.size() * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        return false;   // not cached: a later plan may retry
    }
    for (int rep = 0; rep < 3 && ok; ++rep)
        for (int g : grids) {
            hipError_t e = launch_xcc_probe(g, d, nullptr);
            if (e == hipSuccess) e = hipMemcpy(h.data(), d, g * sizeof(int), hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                ok = false;
                break;
            }
            for (int b0 = 0; b0 + kXCDq <= g && ok; b0 += kXCDq) {
                unsigned seen = 0;
                for (int k = 0; k < kXCDq; ++k) seen |= 1u << (h[b0 + k] & (kXCDq - 1));
                ok = seen == (1u << kXCDq) - 1;
            }
            if (!ok) break;
        }
    (void)hipFree(d);
    (void)hipGetLastError();
    known[device] = ok;
    return ok;
}

// Device records of the hybrid closure iteration: one IterOp per (pass,
// operator) with its neighbours on the lattice, the end-node weights (FP64,
// built on the device), the end-value arrays, and each pass's ev_base.
cfd_status build_iteration(cfd_plan *p, std::vector<PassDesc> &pd, const std::vector<std::array<int, 2>> &pass_tab,
                           const std::vector<int64_t> &toffs) {
    const int nb = (int)p->blocks.size();
    const int bx = p->lat[0], by = p->lat[1];
    auto block_of = [&](int kx, int ky, int kz) { return (kz * by + ky) * bx + kx; };
    // (pass, op) units and their neighbours
    std::map<std::pair<int, int>, int> opidx;
    std::vector<std::pair<int, int>> pops;
    for (size_t i = 0; i < p->passes.size(); ++i)
        for (int o = 0; o < p->passes[i].nops; ++o) {
            if (fused_pass(p->passes[i])) continue;
            opidx[std::make_pair((int)i, o)] = (int)pops.size();
            pops.push_back(std::make_pair((int)i, o));
        }
    auto find_pass = [&](int block, int dir, int op) -> int {
        for (size_t i = 0; i < p->passes.size(); ++i) {
            const PassHost &q = p->passes[i];
            if (q.block != block || q.dir != dir || fused_pass(q)) continue;
            for (int o = 0; o < q.nops; ++o)
                if (q.op[o] == op) return opidx[std::make_pair((int)i, o)];
        }
        return -1;
    };
    // end-node weights per (op scheme, N)
    std::map<std::pair<int, int>, int64_t> wofs;
    std::vector<unsigned char> wspecs;
    int64_t wtotal = 0;
    int maxN = 0;
    std::vector<unsigned char> recs(pops.size() * iter_op_size());
    int64_t ubase = 0;
    int max_units = 0;
    for (size_t u = 0; u < pops.size(); ++u) {
        const int i = pops[u].first, o = pops[u].second;
        const PassHost &ps = p->passes[i];
        const int op = ps.op[o];
        const int b = ps.block;
        const int kx = b % bx, ky = (b / bx) % by, kz = b / (bx * by);
        int km[3] = {kx, ky, kz}, kp[3] = {kx, ky, kz};
        km[ps.dir] = (km[ps.dir] + p->lat[ps.dir] - 1) % p->lat[ps.dir];
        kp[ps.dir] = (kp[ps.dir] + 1) % p->lat[ps.dir];
        const int nm = find_pass(block_of(km[0], km[1], km[2]), ps.dir, op);
        const int np = find_pass(block_of(kp[0], kp[1], kp[2]), ps.dir, op);
        if (nm < 0 || np < 0 || b >= nb) return fail(CFD_EINVAL, "hybrid iteration: neighbour pass not found");
        auto wk = std::make_pair(ps.sch[o], ps.N);
        if (!wofs.count(wk)) {
            wofs[wk] = wtotal;
            const size_t at = wspecs.size();
            wspecs.resize(at + end_weight_spec_size());
            fill_end_weight_spec(wspecs.data() + at, ps.N, p->iter_c, p->base_schemes[ps.sch[o]],
                                 p->schemes[ps.sch[o]], wtotal);
            wtotal += 4 * (int64_t)(ps.N + 2 * kMaxHalf);
            maxN = std::max(maxN, ps.N);
        }
        const int nunits = pd[i].nlines * ps.nfield;
        const int64_t gofs = toffs[pass_tab[i][o]] + table_gvec_offset(ps.P * ps.L, ps.P, ps.nl);
        fill_iter_op(recs.data() + u * iter_op_size(), i, o, nm, np, ubase, nunits, ps.N, p->iter_c, ps.P * ps.L,
                     wofs[wk], gofs, pd[i].hinv[o]);
        pd[i].ev_base[o] = 2 * ubase;
        ubase += nunits;
        max_units = std::max(max_units, nunits);
    }
    const int nw = (int)(wspecs.size() / end_weight_spec_size());
    const size_t es = p->dtype == CFD_F64 ? 8 : 4;
    HIPCHK(dmalloc((void **)&p->d_iops.p, recs.size()));
    HIPCHK(hipMemcpy(p->d_iops.p, recs.data(), recs.size(), hipMemcpyHostToDevice));
    HIPCHK(dmalloc((void **)&p->d_weights.p, std::max<int64_t>(1, wtotal) * sizeof(double)));
    for (DevBuf *bp : {&p->d_ends0, &p->d_endsf, &p->d_ebufA, &p->d_ebufB, &p->d_ev})
        HIPCHK(dmalloc((void **)&bp->p, std::max<int64_t>(1, 2 * ubase) * es));
    {
        void *d_specs = nullptr, *d_scr = nullptr;
        hipError_t e = dmalloc(&d_specs, std::max<size_t>(1, wspecs.size()));
        if (e == hipSuccess) e = dmalloc(&d_scr, (size_t)4 * nw * 2 * maxN * sizeof(double) + 8);
        if (e == hipSuccess) e = hipMemcpy(d_specs, wspecs.data(), wspecs.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_end_weights(nw, d_specs, (double *)p->d_weights.p, (double *)d_scr, maxN, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (d_specs) (void)hipFree(d_specs);
        if (d_scr) (void)hipFree(d_scr);
        if (e != hipSuccess) return hip_fail(e, "building end-node weights");
    }
    p->n_iops = (int)pops.size();
    p->iter_max_units = max_units;
    return CFD_OK;
}

cfd_status build_groups(cfd_plan *p) {
    HIPCHK(hipSetDevice(p->device));
    p->drop_graph();
    if (p->passes.empty()) {   // only biased operators
        p->groups.clear();
        p->nitems = 0;
        return CFD_OK;
    }
    if (p->dtype == CFD_MIXED_BF16) return build_dense(p);
    const bool f32 = p->dtype != CFD_F64;
    // 1. schedule and kernel class of every pass (the fused wave stage's passes
    //    only where their kernel classes exist, and not with iterated closures)
    p->wave_fused_ok = p->wave_fused && p->iter_n == 0;
    for (PassHost &ps : p->passes) {
        if (fused_pass(ps)) {
            ps.cls = nullptr;
            if (!p->wave_fused_ok) continue;
            std::vector<int> cands = candidate_Ps(ps, f32, p->max_lds);
            if (cands.empty()) {
                p->wave_fused_ok = false;
                continue;
            }
            int P = cands[0];
            auto it = p->sched_P.find(std::make_pair(ps.N, ps.dir == 0 ? 1 : 0));
            if (it != p->sched_P.end() && std::find(cands.begin(), cands.end(), it->second) != cands.end())
                P = it->second;
            place_pass(ps, f32, P);
            continue;
        }
        std::vector<int> cands = candidate_Ps(ps, f32, p->max_lds);
        if (cands.empty()) {
            char buf[200];
            std::snprintf(buf, sizeof buf,
                          "no compiled line kernel for N=%d nl=%d nops=%d (stencil half-width %d, direction %d)",
                          ps.N, ps.nl, ps.nops, ps.hw, ps.dir);
            return fail(CFD_EUNSUPPORTED, buf);
        }
        int P = cands[0];
        auto it = p->sched_P.find(std::make_pair(ps.N, ps.dir == 0 ? 1 : 0));
        if (it != p->sched_P.end() && std::find(cands.begin(), cands.end(), it->second) != cands.end())
            P = it->second;
        place_pass(ps, f32, P);
    }
    // 2. tables
    std::map<TabKey, int> tabidx;
    std::vector<TabKey> keys;
    std::vector<int64_t> offs;
    int64_t total = 0;
    std::vector<std::array<int, 2>> pass_tab(p->passes.size());
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const PassHost &ps = p->passes[i];
        if (fused_pass(ps) && !p->wave_fused_ok) {
            pass_tab[i] = {0, 0};
            continue;
        }
        for (int o = 0; o < ps.nops; ++o) {
            TabKey k{ps.sch[o], ps.N, ps.P, ps.L, ps.periodic};
            auto it = tabidx.find(k);
            int id;
            if (it == tabidx.end()) {
                id = (int)keys.size();
                tabidx[k] = id;
                keys.push_back(k);
                offs.push_back(total);
                int64_t n = table_elems(ps.P * ps.L, ps.P, p->schemes[ps.sch[o]].nl);
                total += (n + 7) & ~int64_t(7);
            } else {
                id = it->second;
            }
            pass_tab[i][o] = id;
        }
    }
    std::vector<double> host_tab(total, 0.0);
    std::vector<unsigned char> specs(keys.size() * tabspec_size());
    int64_t scratch_per = 0;
    for (size_t t = 0; t < keys.size(); ++t) {
        const TabKey &k = keys[t];
        const Scheme &s = p->schemes[k.sch];
        fill_coef_block(host_tab.data() + offs[t], s);
        const int L = k.L;
        fill_tabspec(specs.data() + t * tabspec_size(), k.N, k.P, L, s.nl, k.periodic ? 0 : s.nc, k.periodic,
                     s.lhs, offs[t], s.ext, s.cl_d0, s.cl_up, s.gamma);
        scratch_per = std::max<int64_t>(scratch_per, tab_scratch(k.P, L, s.nl));
    }
    p->d_tab64.release();
    p->d_tab32.release();
    p->d_taboff.release();
    HIPCHK(dmalloc((void **)&p->d_tab64.p, total * sizeof(double)));
    HIPCHK(hipMemcpy(p->d_tab64.p, host_tab.data(), total * sizeof(double), hipMemcpyHostToDevice));
    {
        void *d_specs = nullptr, *d_scratch = nullptr, *d_status = nullptr;
        const int ntab = (int)keys.size();
        hipError_t e = dmalloc((void **)&d_specs, specs.size());
        if (e == hipSuccess) e = dmalloc((void **)&d_scratch, std::max<int64_t>(1, scratch_per * ntab) * sizeof(double));
        if (e == hipSuccess) e = dmalloc((void **)&d_status, ntab * sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(d_specs, specs.data(), specs.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_build_tables(ntab, d_specs, (double *)p->d_tab64.p, (double *)d_scratch, scratch_per,
                                    (int *)d_status, nullptr);
        std::vector<int> status(ntab, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(status.data(), d_status, ntab * sizeof(int), hipMemcpyDeviceToHost);
        if (d_specs) (void)hipFree(d_specs);
        if (d_scratch) (void)hipFree(d_scratch);
        if (d_status) (void)hipFree(d_status);
        if (e != hipSuccess) return hip_fail(e, "building solve tables");
        for (int t = 0; t < ntab; ++t)
            if (status[t])
                return fail(CFD_ESINGULAR, "banded system of scheme '" + p->schemes[keys[t].sch].name +
                                               "' cannot be factored without pivoting");
    }
    if (f32) {
        HIPCHK(dmalloc((void **)&p->d_tab32.p, total * sizeof(float)));
        hipError_t e = launch_to_f32(total, (const double *)p->d_tab64.p, (float *)p->d_tab32.p, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "converting tables to FP32");
    }
    HIPCHK(dmalloc((void **)&p->d_taboff.p, std::max<size_t>(1, offs.size()) * sizeof(int64_t)));
    HIPCHK(hipMemcpy(p->d_taboff.p, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice));

    std::vector<PassDesc> pd = pass_descs(p, pass_tab);
    p->release_iteration();
    if (p->iter_n > 0) {
        cfd_status r = build_iteration(p, pd, pass_tab, offs);
        if (r != CFD_OK) return r;
    }
    p->d_pass.release();
    HIPCHK(dmalloc((void **)&p->d_pass.p, std::max<size_t>(1, pd.size()) * sizeof(PassDesc)));
    HIPCHK(hipMemcpy(p->d_pass.p, pd.data(), pd.size() * sizeof(PassDesc), hipMemcpyHostToDevice));

    // 3. stage epilogues of the fused wave stage (d_t phi = Pi, d_t Pi = sum_i
    //    D_i psi_i, d_t psi_i = D_i Pi): D_i Pi updates psi_i, D_y Pi also phi
    //    (k = Pi, its own line value); D_x psi_x and D_y psi_y are stored in
    //    the first launch, and D_z psi_z updates Pi with them as addends in
    //    the second.
    p->d_epi.release();
    if (p->wave_fused_ok) {
        std::vector<EpiDesc> epi(p->passes.size());
        std::memset(epi.data(), 0, epi.size() * sizeof(EpiDesc));
        for (size_t i = 0; i < p->passes.size(); ++i) {
            const PassHost &ps = p->passes[i];
            if (!fused_pass(ps)) continue;
            const cfd_block &b = p->blocks[ps.block];
            const int64_t ng = b.ng, PX = b.n[0] + 2 * ng, PY = b.n[1] + 2 * ng;
            const int64_t npts = (int64_t)b.n[0] * b.n[1] * b.n[2];
            EpiDesc &e = epi[i];
            e.self_tgt = -1;
            e.block = ps.block;
            e.dir = ps.dir;
            for (int d = 0; d < 3; ++d) e.n[d] = b.n[d];
            e.ng = b.ng;
            e.sy = (int32_t)PX;
            e.sz = (int32_t)(PX * PY);
            e.org = ng * (1 + PX + PX * PY);
            const int op = ps.op[0];
            if (op <= 2) {
                e.mode = 1;
                e.tgt = 2 + op;
                if (op == 1) e.self_tgt = 0;
            } else if (op == 5) {
                e.mode = 1;
                e.tgt = 1;
                e.nadd = 2;
                e.add[0] = p->out_off[ps.block] + p->op_slot[3] * npts;
                e.add[1] = p->out_off[ps.block] + p->op_slot[4] * npts;
            }
        }
        HIPCHK(dmalloc((void **)&p->d_epi.p, epi.size() * sizeof(EpiDesc)));
        HIPCHK(hipMemcpy(p->d_epi.p, epi.data(), epi.size() * sizeof(EpiDesc), hipMemcpyHostToDevice));
    }

    // 4. work items.  One launch group per kernel class (x lines optionally in
    //    a group of their own; with concurrent launches, the y/z items of
    //    blocks none of whose y/z lines need LDS also in a group of their own,
    //    whose workgroups then fit on CUs whose LDS the x launch fills);
    //    within a group the items of one block-field are adjacent (x, y, z
    //    passes together) so its input is re-read from cache rather than HBM.
    //    A group's LDS is the most any of its items needs.
    const size_t es = f32 ? 4 : 8;
    std::map<std::pair<const void *, int>, int> gidx;   // (kernel, sub-launch + 4 iomode)
    std::vector<std::vector<WorkItem>> gitems;
    std::vector<std::vector<int>> gbf;        // block-field of each item
    std::vector<std::vector<int64_t>> gcost;  // rows x lines of each item
    std::vector<Group> groups;
    std::vector<std::vector<int>> by_block(p->blocks.size());
    for (size_t i = 0; i < p->passes.size(); ++i) by_block[p->passes[i].block].push_back((int)i);
    for (size_t b = 0; b < p->blocks.size(); ++b) {
        // the LDS-free y/z launch takes a block only if none of its y/z passes
        // needs LDS, so a block-field's y and z lines stay in one launch
        bool yz_lds_free = true;
        for (int i : by_block[b]) {
            const PassHost &ps = p->passes[i];
            if (fused_pass(ps)) continue;
            if (ps.dir != 0 && exch_bytes(ps.nl, ps.nops, ps.P, ps.periodic, es) > 0) yz_lds_free = false;
        }
        for (int f = 0; f < p->nfields; ++f) {
            for (int i : by_block[b]) {
                const PassHost &ps = p->passes[i];
                if (f < ps.field0 || f >= ps.field0 + ps.nfield) continue;
                if (fused_pass(ps) && !p->wave_fused_ok) continue;
                const size_t lds = pass_lds(ps, f32);
                int sub = 0;
                if (p->split_x && ps.dir == 0) sub = 1;
                else if (p->split_x && p->concurrent && yz_lds_free) sub = 2;
                auto key = std::make_pair(ps.cls->fn, sub + 4 * ps.iomode);
                auto it = gidx.find(key);
                int gi;
                if (it == gidx.end()) {
                    gi = (int)groups.size();
                    gidx[key] = gi;
                    Group g;
                    g.fn = ps.cls->fn;
                    g.wg = ps.cls->wg;
                    g.lds = 0;
                    g.iomode = ps.iomode;
                    groups.push_back(g);
                    gitems.emplace_back();
                    gbf.emplace_back();
                    gcost.emplace_back();
                } else {
                    gi = it->second;
                }
                groups[gi].lds = std::max(groups[gi].lds, lds);
                const int per_item = kWave * (waves_for(ps.P) / ps.P);
                const int meta = ps.P | (ps.lcode << 4) | ((ps.C - 1) << 8);
                for (int l0 = 0; l0 < pd[i].nlines; l0 += per_item) {
                    gitems[gi].push_back(WorkItem{(int32_t)i, f - ps.field0, l0, meta});
                    gbf[gi].push_back((int)(b * p->nfields + f));
                    gcost[gi].push_back((int64_t)per_item * ps.P * ps.L);
                }
            }
        }
    }
    // XCD-aware modes: block-fields are dealt to kXCDq queues (least-loaded
    // first, by the cost of all their passes in every group), the same way for
    // every group, so a block-field's x, y and z lines, also in separate
    // launches, share one XCD's L2.  Workgroup b runs on XCD b mod kXCDq.
    const int nbf = (int)(p->blocks.size() * p->nfields);
    std::vector<int> bf_queue(nbf, 0);
    if (p->xcd) {
        std::vector<int64_t> bf_cost(nbf, 0);
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            if (fused_iomode(groups[gi].iomode)) continue;   // the fused stage's copies follow the same queues
            for (size_t e = 0; e < gitems[gi].size(); ++e) bf_cost[gbf[gi][e]] += gcost[gi][e];
        }
        std::vector<int64_t> load(kXCDq, 0);
        for (int bf = 0; bf < nbf; ++bf) {
            if (!bf_cost[bf]) continue;
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            bf_queue[bf] = k;
            load[k] += bf_cost[bf];
        }
    }
    std::vector<WorkItem> items;
    std::vector<int> qoffs;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group &g = groups[gi];
        g.item0 = (int64_t)items.size();
        g.nitems = (int64_t)gitems[gi].size();
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, g.fn, kWave * g.wg, g.lds) != hipSuccess || nb < 1)
            nb = 1;
        (void)hipGetLastError();
        g.grid_persist = (int)std::min<int64_t>(g.nitems, (int64_t)nb * p->cus);
        g.qoff_index = -1;
        if (p->xcd && g.nitems >= 8 * kXCDq && (p->persistent || p->xcd_interleave_ok)) {
            std::vector<std::vector<WorkItem>> q(kXCDq);
            for (size_t e = 0; e < gitems[gi].size(); ++e) q[bf_queue[gbf[gi][e]]].push_back(gitems[gi][e]);
            if (p->persistent) {
                // persistent grid: workgroup b walks queue b mod kXCDq
                g.qoff_index = (int)qoffs.size();
                int off = 0;
                for (int k = 0; k < kXCDq; ++k) {
                    qoffs.push_back(off);
                    off += (int)q[k].size();
                    items.insert(items.end(), q[k].begin(), q[k].end());
                }
                qoffs.push_back(off);
                g.grid_persist = std::max(kXCDq, (g.grid_persist / kXCDq) * kXCDq);
            } else {
                // one workgroup per item: queue k's items at positions k, k + kXCDq, ...;
                // shorter queues are padded with empty items (pass -1)
                size_t len = 0;
                for (auto &v : q) len = std::max(len, v.size());
                for (size_t r = 0; r < len; ++r)
                    for (int k = 0; k < kXCDq; ++k)
                        items.push_back(r < q[k].size() ? q[k][r] : WorkItem{-1, 0, 0, 0});
                g.nitems = (int64_t)(items.size() - g.item0);
                g.grid_persist = (int)std::min<int64_t>(g.nitems, (int64_t)nb * p->cus);
                g.qoff_index = (int)qoffs.size();   // marker: workgroups pick their XCD's item
                qoffs.push_back(-1);
            }
        } else {
            items.insert(items.end(), gitems[gi].begin(), gitems[gi].end());
        }
    }
    p->groups = groups;
    p->d_qoff.release();
    if (!qoffs.empty()) {
        HIPCHK(dmalloc((void **)&p->d_qoff.p, qoffs.size() * sizeof(int)));
        HIPCHK(hipMemcpy(p->d_qoff.p, qoffs.data(), qoffs.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    p->nitems = (int64_t)items.size();
    p->d_items.release();
    HIPCHK(dmalloc((void **)&p->d_items.p, std::max<size_t>(1, items.size()) * sizeof(WorkItem)));
    HIPCHK(hipMemcpy(p->d_items.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    return CFD_OK;
}


// Dense mixed-precision plans: periodic lines only, one operator per pass,
// tables formed in FP64 on the GPU (A^-1 B and A^-1 by Gauss-Jordan).
cfd_status build_dense(cfd_plan *p) {
    std::map<std::pair<int, int>, int> tabidx;   // (scheme, N) -> table
    std::vector<std::pair<int, int>> keys;
    std::vector<int64_t> offs;
    int64_t total = 0;
    std::vector<std::array<int, 2>> pass_tab(p->passes.size());
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const PassHost &ps = p->passes[i];
        auto k = std::make_pair(ps.sch[0], ps.N);
        auto it = tabidx.find(k);
        int id;
        if (it == tabidx.end()) {
            id = (int)keys.size();
            tabidx[k] = id;
            keys.push_back(k);
            offs.push_back(total);
            total += (int64_t)((dense_tab_bytes(ps.N) + 255) & ~size_t(255));
        } else {
            id = it->second;
        }
        pass_tab[i] = {id, id};
    }
    const int ntab = (int)keys.size();
    std::vector<unsigned char> specs(ntab * dense_tab_struct_size());
    std::vector<double> coefs(ntab * 16, 0.0);
    int64_t scratch_per = 0;
    for (int t = 0; t < ntab; ++t) {
        const Scheme &s = p->schemes[keys[t].first];
        const int N = keys[t].second;
        fill_dense_tab(specs.data() + t * dense_tab_struct_size(), N, s.nl, s.m, offs[t]);
        for (int m = 0; m < 11; ++m) coefs[t * 16 + m] = s.rhs[m];
        for (int j = 0; j < 5; ++j) coefs[t * 16 + 11 + j] = s.lhs[j];
        scratch_per = std::max<int64_t>(scratch_per, (int64_t)N * 3 * N);
    }
    p->d_dense.release();
    p->d_dense_specs.release();
    HIPCHK(dmalloc((void **)&p->d_dense.p, std::max<int64_t>(total, 256)));
    HIPCHK(dmalloc((void **)&p->d_dense_specs.p, specs.size()));
    HIPCHK(hipMemcpy(p->d_dense_specs.p, specs.data(), specs.size(), hipMemcpyHostToDevice));
    {
        void *d_coefs = nullptr, *d_scratch = nullptr, *d_status = nullptr;
        hipError_t e = dmalloc((void **)&d_coefs, coefs.size() * sizeof(double));
        if (e == hipSuccess) e = dmalloc((void **)&d_scratch, scratch_per * ntab * sizeof(double));
        if (e == hipSuccess) e = dmalloc((void **)&d_status, ntab * sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(d_coefs, coefs.data(), coefs.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_dense_form(ntab, p->d_dense_specs.p, (const double *)d_coefs, (unsigned char *)p->d_dense.p,
                                  (double *)d_scratch, scratch_per, (int *)d_status, nullptr);
        std::vector<int> status(ntab, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(status.data(), d_status, ntab * sizeof(int), hipMemcpyDeviceToHost);
        if (d_coefs) (void)hipFree(d_coefs);
        if (d_scratch) (void)hipFree(d_scratch);
        if (d_status) (void)hipFree(d_status);
        if (e != hipSuccess) return hip_fail(e, "forming the dense periodic operator");
        for (int t = 0; t < ntab; ++t)
            if (status[t]) return fail(CFD_ESINGULAR, "periodic operator matrix is singular");
    }
    std::vector<PassDesc> pd = pass_descs(p, pass_tab);
    for (const PassDesc &q : pd)   // the kernel addresses a field with 32-bit byte offsets
        if (q.in_fstride * 4 >= (int64_t(1) << 32) || q.out_fstride * 4 >= (int64_t(1) << 32))
            return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: a field exceeds 4 GiB");
    p->d_pass.release();
    HIPCHK(dmalloc((void **)&p->d_pass.p, std::max<size_t>(1, pd.size()) * sizeof(PassDesc)));
    HIPCHK(hipMemcpy(p->d_pass.p, pd.data(), pd.size() * sizeof(PassDesc), hipMemcpyHostToDevice));
    // work items: dense_item_lines() lines of one pass and field; one group
    // (kernel) per (N, x or not).  Items of one table are kept together: a
    // workgroup stages the table's circulant blocks in LDS once for them
    std::map<std::array<int, 3>, std::vector<std::array<int, 4>>> by_class_t;   // (tab, pass, field, line0)
    const size_t isz = dense_item_size();
    for (size_t b = 0; b < p->blocks.size(); ++b)
        for (int f = 0; f < p->nfields; ++f)
            for (size_t i = 0; i < p->passes.size(); ++i) {
                const PassHost &ps = p->passes[i];
                if (ps.block != (int)b || f < ps.field0 || f >= ps.field0 + ps.nfield) continue;
                const int xd = (pd[i].sd == 1 && pd[i].osd == 1) ? 1 : 0;
                const int wide = p->schemes[ps.sch[0]].m > 3 ? 1 : 0;
                auto &v = by_class_t[{ps.N, xd, wide}];
                for (int l0 = 0; l0 < pd[i].nlines; l0 += dense_item_lines())
                    v.push_back({pass_tab[i][0], (int)i, f - ps.field0, l0});
            }
    std::map<std::array<int, 3>, std::vector<unsigned char>> by_class;
    for (auto &kv : by_class_t) {
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [](const std::array<int, 4> &x, const std::array<int, 4> &y) { return x[0] < y[0]; });
        std::vector<unsigned char> &items = by_class[kv.first];
        items.resize(kv.second.size() * isz);
        for (size_t e = 0; e < kv.second.size(); ++e) {
            const auto &t = kv.second[e];
            fill_dense_item(items.data() + e * isz, t[1], t[2], t[3], t[0]);
        }
    }
    std::vector<unsigned char> items;
    p->groups.clear();
    for (auto &kv : by_class) {
        Group g;
        g.fn = dense_apply_fn(kv.first[0], kv.first[1] != 0, kv.first[2] != 0);
        if (!g.fn) return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: unsupported line length");
        g.lds = 0;
        g.item0 = (int64_t)(items.size() / isz);
        g.nitems = (int64_t)(kv.second.size() / isz);
        int per_cu = 1;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, g.fn, 256, 0));
        g.grid_persist = (int)std::min<int64_t>(g.nitems, (int64_t)p->cus * std::max(1, per_cu));
        items.insert(items.end(), kv.second.begin(), kv.second.end());
        p->groups.push_back(g);
    }
    p->nitems = (int64_t)(items.size() / isz);
    p->d_items.release();
    HIPCHK(dmalloc((void **)&p->d_items.p, std::max<size_t>(1, items.size())));
    HIPCHK(hipMemcpy(p->d_items.p, items.data(), items.size(), hipMemcpyHostToDevice));
    return CFD_OK;
}

// Biased (upwind) operators: one BiasPass per (block, operator) over the
// fields the operator selects, work items of 64 lines per (pass, field),
// grouped by stencil half-width class; coefficient records in the plan's
// element type.  Independent of the schedule, built once at plan creation.
cfd_status build_biased(cfd_plan *p) {
    const bool f32 = p->dtype != CFD_F64;
    std::vector<int> bops;
    for (size_t o = 0; o < p->ops.size(); ++o)
        if (p->schemes[o].kind == 1) bops.push_back((int)o);
    p->bgroups.clear();
    p->nbitems = 0;
    if (bops.empty()) return CFD_OK;
    std::vector<double> rec64(bops.size() * kBiasRec, 0.0);
    for (size_t i = 0; i < bops.size(); ++i) {
        const Scheme &s = p->schemes[bops[i]];
        double *r = rec64.data() + i * kBiasRec;
        r[0] = s.balpha;
        for (int m = 0; m < 2 * kBiasHalf + 1; ++m) r[1 + m] = s.ba[m];
        for (int m = 0; m < 2 * kBiasHalf + 2; ++m) r[12 + m] = s.bc[m];
        r[24] = 1.0 / (1.0 - s.balpha * s.balpha);
        double pw = 1.0;
        for (int n = 0; n <= kBiasMaxPN; ++n, pw *= -s.balpha) r[kBiasPow + n] = pw;
    }
    std::vector<BiasPass> bp;
    int64_t ev_total = 0;
    p->bpinfo.clear();
    // kernel class (hb, L, x lines) -> items; L = 0 is the sweep kernel
    std::map<std::array<int, 3>, std::vector<BiasItem>> by_cls;
    std::map<std::array<int, 3>, size_t> cls_lds;
    std::map<std::array<int, 3>, std::vector<int>> by_unit;   // first item of each unit
    for (size_t b = 0; b < p->blocks.size(); ++b) {
        const cfd_block &bl = p->blocks[b];
        const int64_t npts = (int64_t)bl.n[0] * bl.n[1] * bl.n[2];
        for (size_t i = 0; i < bops.size(); ++i) {
            const int o = bops[i];
            const Scheme &s = p->schemes[o];
            const cfd_op &op = p->ops[o];
            PassHost ph;
            ph.dir = op.dir;
            ph.N = bl.n[op.dir];
            ph.periodic = bl.boundary[op.dir] == CFD_BOUNDARY_PERIODIC;
            PassDesc d;
            const int64_t ob[2] = {p->out_off[b] + p->op_slot[o] * npts, 0};
            const int tab[2] = {0, 0};
            const double hi[2] = {0, 0};
            fill_pass_desc(d, bl, p->in_off[b], ph, ob, tab, hi);
            BiasPass q;
            std::memset(&q, 0, sizeof q);
            q.in_base = d.in_base;
            q.in_fstride = d.in_fstride;
            q.vel_base = (s.bias == 0) ? d.in_base + (int64_t)op.vel_field * d.in_fstride : 0;
            // items carry the input field index; a one-field operator's output
            // slot holds that field at index 0
            q.out_fstride = d.out_fstride;
            q.out_base = d.out_base[0] - (op.field < 0 ? 0 : (int64_t)op.field * d.out_fstride);
            q.su = d.su;
            q.sv = d.sv;
            q.sd = d.sd;
            q.osu = d.osu;
            q.osv = d.osv;
            q.osd = d.osd;
            q.nu = d.nu;
            q.nlines = d.nlines;
            q.N = d.N;
            q.ng = bl.ng;
            q.periodic = ph.periodic;
            q.mode = s.bias;
            q.tab = (int)i;
            q.hb = s.bhalf < 2 ? 2 : s.bhalf;
            q.hinv = 1.0 / bl.h[op.dir];
            q.wrap = 1.0 / (1.0 - std::pow(-s.balpha, (double)d.N));
            q.ev_base = ev_total;
            q.s2 = nullptr;
            q.s2_base = q.s2f = 0;
            q.s2u = q.s2v = q.s2d = q.s2_in = 0;
            q.w2 = q.w2c = 0.0;
            const double h2 = bl.h[op.dir] * bl.h[op.dir];
            if (p->emb_sch[o] >= 0) {   // W: the embedded pass's result in scratch
                const int f0e = op.field < 0 ? 0 : op.field;
                q.s2 = p->d_mscr.p;
                q.s2_base = p->emb_off.at(std::make_pair((int)b, o)) - (int64_t)f0e * npts;
                q.s2f = d.out_fstride;
                q.s2u = d.osu;
                q.s2v = d.osv;
                q.s2d = d.osd;
                q.w2 = s.ba2 * h2;
            } else if (s.hermite) {     // U: the sampled f'' field of the input
                q.s2_in = 1;
                q.s2_base = d.in_base + (int64_t)op.aux_field * d.in_fstride;
                q.s2u = d.su;
                q.s2v = d.sv;
                q.s2d = d.sd;
                q.w2 = s.ba2 * h2;
                q.w2c = s.bc2 * h2;
            }
            if (!biased_supported(q.hb)) return fail(CFD_EUNSUPPORTED, "biased stencil half-width not compiled");
            const int pi = (int)bp.size();
            bp.push_back(q);
            const int64_t entries = (int64_t)p->nfields * q.nlines;
            p->bpinfo.push_back({(int64_t)b, (int64_t)o, ev_total, entries});
            ev_total += entries;
            const int f0 = op.field < 0 ? 0 : op.field;
            const int nf = op.field < 0 ? p->nfields : 1;
            // partitions: every partition keeps at least two rows ((P-1) ceil(N/P) <= N - 2)
            const int N = q.N;
            // (at most 12 rows per partition where 4 partitions allow it: fewer registers)
            const int P = (N <= 12) ? 1 : (N <= 24) ? 2 : (N <= kBiasMaxPN) ? 4 : 0;
            const int Lr = P ? (N + P - 1) / P : 0;
            const int L = P == 0 ? 0 : (Lr <= 8 ? 8 : Lr <= 12 ? 12 : 16);
            const int xdir = (P > 0 && op.dir == 0) ? 1 : 0;
            const std::array<int, 3> key{q.hb, L, xdir};
            const int step = P ? kWave * (4 / P) : kWave;
            size_t lds = biased_lds(p->dtype != CFD_F64, q.hb, L, xdir, P ? P : 1, N);
            size_t &cl = cls_lds[key];
            cl = std::max(cl, lds);
            // unit = the items of one line group over all selected fields (they share the velocity)
            for (int l0 = 0; l0 < q.nlines; l0 += step) {
                by_unit[key].push_back((int)by_cls[key].size());
                for (int f = 0; f < nf; ++f) by_cls[key].push_back(BiasItem{pi, f0 + f, l0, P});
            }
        }
    }
    // Where the device deals workgroups round-robin over its 8 XCDs, a line
    // group's items (all its fields) go to one XCD: units are dealt to XCDs in
    // turn and position 8 r + x holds XCD x's r-th item, queues padded with
    // empty items, so the velocity lines stay in that XCD's L2.
    if (p->xcd_interleave_ok) {
        for (auto &kv : by_cls) {
            if (kv.first[1] == 0) continue;   // sweep kernel: four items per workgroup, plain order
            const std::vector<int> &u0 = by_unit[kv.first];
            std::vector<std::vector<BiasItem>> q(kXCDq);
            for (size_t ui = 0; ui < u0.size(); ++ui) {
                const int b0 = u0[ui], b1 = (ui + 1 < u0.size()) ? u0[ui + 1] : (int)kv.second.size();
                for (int i = b0; i < b1; ++i) q[ui % kXCDq].push_back(kv.second[i]);
            }
            size_t len = 0;
            for (auto &v : q) len = std::max(len, v.size());
            std::vector<BiasItem> inter(len * kXCDq, BiasItem{-1, 0, 0, 0});
            for (int x = 0; x < kXCDq; ++x)
                for (size_t r = 0; r < q[x].size(); ++r) inter[r * kXCDq + x] = q[x][r];
            kv.second.swap(inter);
        }
    }
    std::vector<BiasItem> items;
    for (auto &kv : by_cls) {
        cfd_plan::BGroup g;
        g.hb = kv.first[0];
        g.L = kv.first[1];
        g.xdir = kv.first[2];
        g.lds = cls_lds[kv.first];
        if (g.lds > p->max_lds) return fail(CFD_EUNSUPPORTED, "biased-line tile exceeds the device's LDS");
        g.item0 = (int64_t)items.size();
        g.nitems = (int64_t)kv.second.size();
        items.insert(items.end(), kv.second.begin(), kv.second.end());
        p->bgroups.push_back(g);
    }
    p->nbitems = (int64_t)items.size();
    p->bev_entries = ev_total;
    if (p->nbitems > INT32_MAX) return fail(CFD_EUNSUPPORTED, "too many biased work items");
    HIPCHK(dmalloc((void **)&p->d_bpass.p, bp.size() * sizeof(BiasPass)));
    HIPCHK(hipMemcpy(p->d_bpass.p, bp.data(), bp.size() * sizeof(BiasPass), hipMemcpyHostToDevice));
    HIPCHK(dmalloc((void **)&p->d_bitems.p, items.size() * sizeof(BiasItem)));
    HIPCHK(hipMemcpy(p->d_bitems.p, items.data(), items.size() * sizeof(BiasItem), hipMemcpyHostToDevice));
    if (f32) {
        std::vector<float> rec32(rec64.begin(), rec64.end());
        HIPCHK(dmalloc((void **)&p->d_bcoef.p, rec32.size() * sizeof(float)));
        HIPCHK(hipMemcpy(p->d_bcoef.p, rec32.data(), rec32.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
        HIPCHK(dmalloc((void **)&p->d_bcoef.p, rec64.size() * sizeof(double)));
        HIPCHK(hipMemcpy(p->d_bcoef.p, rec64.data(), rec64.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return CFD_OK;
}

// One launch per biased kernel class; in the concurrent mode every class after
// the first on a forked stream (the classes write disjoint outputs), joined
// before the caller's stream goes on.
cfd_status launch_biased_groups(cfd_plan *p, const void *in, void *out, hipStream_t st, const void *ev = nullptr,
                                void *ends = nullptr) {
    const size_t n = p->bgroups.size();
    const bool fork = p->bconcurrent && n > 1 && p->aux.size() + 1 >= n && p->ev.size() >= n;
    if (fork) HIPCHK(hipEventRecord(p->ev[0], st));
    for (size_t i = 0; i < n; ++i) {
        const cfd_plan::BGroup &g = p->bgroups[i];
        hipStream_t s = (fork && i > 0) ? p->aux[i - 1] : st;
        if (s != st) HIPCHK(hipStreamWaitEvent(s, p->ev[0], 0));
        hipError_t e = launch_biased(p->dtype != CFD_F64, g.hb, g.L, g.xdir, g.lds,
                                     (const BiasItem *)p->d_bitems.p + g.item0, (int)g.nitems,
                                     (const BiasPass *)p->d_bpass.p, p->d_bcoef.p, in, out, ev, ends, s);
        if (e != hipSuccess) return hip_fail(e, "launching the biased-line kernel");
        if (s != st) HIPCHK(hipEventRecord(p->ev[i], s));
    }
    if (fork)
        for (size_t i = 1; i < n; ++i) HIPCHK(hipStreamWaitEvent(st, p->ev[i], 0));
    return CFD_OK;
}

cfd_status launch_group(cfd_plan *p, const Group &g, const void *in, void *out, hipStream_t st,
                        const RkArgs *rk = nullptr) {
    const int grid = p->persistent ? g.grid_persist : (int)g.nitems;
    if (g.iomode == 1) out = p->d_mscr.p;
    if (g.iomode == 5 || g.iomode == 6) in = p->d_mscr.p;
    if (g.iomode == 2) {
        in = p->d_mscr.p;
        out = p->d_mscr.p;
    }
    hipError_t e;
    if (p->dtype == CFD_MIXED_BF16) {
        e = launch_dense_apply(g.fn, grid, st, (const unsigned char *)p->d_items.p + g.item0 * dense_item_size(),
                               (int)g.nitems, (const PassDesc *)p->d_pass.p, p->d_dense_specs.p,
                               (const unsigned char *)p->d_dense.p, (const float *)in, (float *)out);
    } else {
        const void *tabs = (p->dtype == CFD_F64) ? p->d_tab64.p : p->d_tab32.p;
        const int *qoff = (g.qoff_index >= 0) ? (const int *)p->d_qoff.p + g.qoff_index : nullptr;
        e = launch_lines(g.fn, g.wg, grid, g.lds, st, (const WorkItem *)p->d_items.p + g.item0, (int)g.nitems, qoff,
                         (const PassDesc *)p->d_pass.p, tabs, (const int64_t *)p->d_taboff.p, in, out,
                         p->iter_n > 0 ? p->d_ev.p : nullptr, rk);
    }
    if (e != hipSuccess) return hip_fail(e, "launching a kernel group");
    return CFD_OK;
}

// Streams and events of the concurrent mode, made outside any capture.
cfd_status ensure_aux(cfd_plan *p) {
    const size_t ng = std::max(p->groups.size(), p->bgroups.size());
    const size_t need = ng > 1 ? ng - 1 : 0;
    while (p->aux.size() < need) {
        hipStream_t s;
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        p->aux.push_back(s);
    }
    while (p->ev.size() < need + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->ev.push_back(e);
    }
    return CFD_OK;
}

// Block layout on the device, read by the ghost exchange and the stage
// kernels: input and output offsets per block, and per block (nx, ny, nz, ng)
// followed by the first 64-node piece (of the interior, x fastest) of each
// block and their total.
// Uploaded once at plan creation, so those calls allocate nothing.
cfd_status upload_layout(cfd_plan *p) {
    const int nb = (int)p->blocks.size();
    std::vector<int> sh(4 * nb + nb + 1);
    int64_t units = 0;
    for (int b = 0; b < nb; ++b) {
        const cfd_block &bl = p->blocks[b];
        sh[4 * b] = bl.n[0];
        sh[4 * b + 1] = bl.n[1];
        sh[4 * b + 2] = bl.n[2];
        sh[4 * b + 3] = bl.ng;
        sh[4 * nb + b] = (int)std::min<int64_t>(units, INT32_MAX);
        units += ((int64_t)bl.n[0] * bl.n[1] * bl.n[2] + 63) / 64;
    }
    sh[4 * nb + nb] = (int)std::min<int64_t>(units, INT32_MAX);
    p->nunits = units;
    HIPCHK(dmalloc((void **)&p->d_shapes.p, sh.size() * sizeof(int)));
    HIPCHK(hipMemcpy(p->d_shapes.p, sh.data(), sh.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(dmalloc((void **)&p->d_outoff.p, nb * sizeof(int64_t)));
    HIPCHK(hipMemcpy(p->d_outoff.p, p->out_off.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(dmalloc((void **)&p->d_inoff.p, nb * sizeof(int64_t)));
    HIPCHK(hipMemcpy(p->d_inoff.p, p->in_off.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(dmalloc((void **)&p->d_hpairs.p, (size_t)18 * nb * sizeof(int)));
    HIPCHK(dmalloc((void **)&p->d_vpairs.p, (size_t)6 * nb * sizeof(int)));
    return CFD_OK;
}

// Device tables, work lists and launch groups for the current schedule.
cfd_status build(cfd_plan *p) {
    cfd_status r = build_groups(p);
    if (r == CFD_OK) r = ensure_aux(p);
    return r;
}

// Hybrid closure iteration, before the line kernels: end-node values of
// iterate 0 and of the zero-end-value solutions, iter_n - 1 exchange steps,
// then every line's end values for the last iterate (into d_ev).
cfd_status enqueue_iteration(cfd_plan *p, const void *in, hipStream_t st) {
    const int f32 = p->dtype != CFD_F64;
    hipError_t e = launch_end_values(f32, p->n_iops, p->iter_max_units, p->d_iops.p, (const PassDesc *)p->d_pass.p,
                                     (const double *)p->d_weights.p, in, p->d_ends0.p, p->d_endsf.p, st);
    const void *prev = p->d_ends0.p;
    for (int i = 1; i < p->iter_n && e == hipSuccess; ++i) {
        void *next = (i % 2) ? p->d_ebufA.p : p->d_ebufB.p;
        e = launch_iter_ends(f32, p->n_iops, p->iter_max_units, p->d_iops.p, (const double *)p->d_tab64.p,
                             p->d_endsf.p, prev, next, 0, st);
        prev = next;
    }
    if (e == hipSuccess)
        e = launch_iter_ends(f32, p->n_iops, p->iter_max_units, p->d_iops.p, (const double *)p->d_tab64.p,
                             p->d_endsf.p, prev, p->d_ev.p, 1, st);
    if (e != hipSuccess) return hip_fail(e, "launching the closure iteration");
    return CFD_OK;
}

cfd_status enqueue(cfd_plan *p, const void *in, void *out, hipStream_t st) {
    if (p->iter_n > 0 && p->n_iops > 0) {
        cfd_status r = enqueue_iteration(p, in, st);
        if (r != CFD_OK) return r;
    }
    auto biased = [&]() -> cfd_status {
        if (p->nbitems > 0 && p->iter_n > 0 && p->d_bev.p) {
            // iterated biased closures: iterate [0] writes every line's end values,
            // each later iterate enters with its neighbours' (Eq. iter_left_X)
            cfd_status r = launch_biased_groups(p, in, out, st, nullptr, p->d_bends.p);
            for (int i = 1; i <= p->iter_n && r == CFD_OK; ++i) {
                hipError_t e = launch_bias_gather(p->dtype != CFD_F64, (int)p->bpinfo.size(), p->bev_max,
                                                  (const int64_t *)p->d_bgrecs.p, p->d_bends.p, p->d_bev.p, st);
                if (e != hipSuccess) return hip_fail(e, "launching the biased end-value gather");
                r = launch_biased_groups(p, in, out, st, p->d_bev.p, p->d_bends.p);
            }
            return r;
        }
        if (p->nbitems > 0) return launch_biased_groups(p, in, out, st);
        return CFD_OK;
    };
    // W operators read the second derivative stage 0 leaves in the scratch
    const bool biased_late = !p->emb_off.empty();
    if (!biased_late) {
        cfd_status r = biased();
        if (r != CFD_OK) return r;
    }
    // stage 0: every group reading the input; stage 1: the second stage of the
    // mixed derivatives (reads what stage 0 left in the scratch; the first
    // order stores into the output); stage 2: the second order adds to it
    for (int stage = 0; stage < 3; ++stage) {
        if (stage == 1 && biased_late) {
            cfd_status r = biased();
            if (r != CFD_OK) return r;
        }
        std::vector<const Group *> act;
        for (const Group &g : p->groups)
            if (g.nitems > 0 && !fused_iomode(g.iomode) && apply_stage(g.iomode) == stage) act.push_back(&g);
        if (p->concurrent && act.size() > 1 && p->aux.size() + 1 >= act.size() && p->ev.size() >= act.size()) {
            // fork: every group after the first on its own stream, all ordered after
            // the caller's earlier work; join: the caller's stream waits for all
            HIPCHK(hipEventRecord(p->ev[0], st));
            for (size_t i = 1; i < act.size(); ++i) {
                HIPCHK(hipStreamWaitEvent(p->aux[i - 1], p->ev[0], 0));
                cfd_status r = launch_group(p, *act[i], in, out, p->aux[i - 1]);
                if (r != CFD_OK) return r;
                HIPCHK(hipEventRecord(p->ev[i], p->aux[i - 1]));
            }
            cfd_status r = launch_group(p, *act[0], in, out, st);
            if (r != CFD_OK) return r;
            for (size_t i = 1; i < act.size(); ++i) HIPCHK(hipStreamWaitEvent(st, p->ev[i], 0));
        } else {
            for (const Group *g : act) {
                cfd_status r = launch_group(p, *g, in, out, st);
                if (r != CFD_OK) return r;
            }
        }
    }
    return CFD_OK;
}

// The fused wave stage: the first launch (iomode 3) updates phi and psi and
// stores D_x psi_x, D_y psi_y into work; the second (iomode 4), after it on
// the same stream, updates Pi.
cfd_status enqueue_wave_fused(cfd_plan *p, const void *src, void *work, const RkArgs &rk, hipStream_t st) {
    for (int mode = 3; mode <= 4; ++mode)
        for (const Group &g : p->groups) {
            if (g.iomode != mode || g.nitems == 0) continue;
            cfd_status r = launch_group(p, g, src, work, st, &rk);
            if (r != CFD_OK) return r;
        }
    return CFD_OK;
}

// Apply the plan with its current schedule into out_dev, and with the plain
// persistent grid (same partitions, no XCD order, no split, sequential) into
// a temporary buffer; same = every 32-bit word of the two outputs agrees.
// Both buffers are first filled with the same pattern, so output words no
// item writes (gaps between explicitly placed blocks) compare equal.
cfd_status same_as_plain(cfd_plan *p, const void *in_dev, void *out_dev, hipStream_t st, bool &same) {
    const size_t bytes = (size_t)p->out_elems * elem_size(p->dtype);
    same = true;
    if (bytes == 0) return CFD_OK;
    void *tmp = nullptr;
    unsigned long long *cnt = nullptr;
    hipError_t e = dmalloc(&tmp, bytes);
    if (e == hipSuccess) e = dmalloc((void **)&cnt, sizeof(unsigned long long));
    if (e != hipSuccess) {
        if (tmp) (void)hipFree(tmp);
        return hip_fail(e, "autotune check buffer");
    }
    const bool pe = p->persistent, xc = p->xcd, sx = p->split_x, cc = p->concurrent;
    cfd_status r = CFD_OK;
    e = hipMemsetAsync(out_dev, 0x7f, bytes, st);
    if (e == hipSuccess) e = hipMemsetAsync(tmp, 0x7f, bytes, st);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) r = hip_fail(e, "autotune check fill");
    if (r == CFD_OK) r = enqueue(p, in_dev, out_dev, st);
    if (r == CFD_OK) {
        p->persistent = true;
        p->xcd = p->split_x = p->concurrent = false;
        r = build(p);
        if (r == CFD_OK) r = enqueue(p, in_dev, tmp, st);
        p->persistent = pe;
        p->xcd = xc;
        p->split_x = sx;
        p->concurrent = cc;
        cfd_status r2 = build(p);
        if (r == CFD_OK) r = r2;
    }
    unsigned long long diff = 0;
    if (r == CFD_OK) {
        e = launch_count_diff((int64_t)(bytes / 4), out_dev, tmp, cnt, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&diff, cnt, sizeof diff, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = hip_fail(e, "autotune check");
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(tmp);
    (void)hipFree(cnt);
    same = diff == 0;
    return r;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int cfd_abi_version(void) { return CFD_ABI_VERSION; }

const char *cfd_last_error(void) { return g_err.c_str(); }

cfd_status cfd_scheme_named(const char *name, cfd_scheme **out) {
    if (!name || !out) return fail(CFD_EINVAL, "cfd_scheme_named: null argument");
    Scheme s;
    std::string err;
    cfd_status st = scheme_from_name(name, s, err);
    if (st != CFD_OK) return fail(st, err);
    *out = new cfd_scheme{s};
    return CFD_OK;
}

cfd_status cfd_scheme_design(int d, int order, int nl, int m, double eta_c, int closure_mc, int matched,
                             cfd_scheme **out) {
    if (!out) return fail(CFD_EINVAL, "cfd_scheme_design: null output");
    Scheme s;
    std::string err;
    cfd_status st = design_centred(d, order, nl, m, eta_c, closure_mc, matched, s, err);
    if (st != CFD_OK) return fail(st, err);
    if (nl > 0 && closure_mc == 0) s.nc = 0;
    char buf[96];
    std::snprintf(buf, sizeof buf, "design(d=%d,order=%d,nl=%d,m=%d,eta_c=%g,mc=%d,%s)", d, order, nl, m, eta_c,
                  closure_mc, matched ? "matched" : "order-only");
    s.name = buf;
    *out = new cfd_scheme{s};
    return CFD_OK;
}

cfd_status cfd_scheme_create(int d, int order, int nl, const double *lhs, int m, const double *rhs, int nc, int mc,
                             const double *closure, cfd_scheme **out) {
    if (!out || !lhs || !rhs) return fail(CFD_EINVAL, "cfd_scheme_create: null argument");
    if (d < 1 || d > 2 || order < 1 || nl < 0 || nl > kMaxNL || m < 0 || m > kMaxHalf || mc < 0 || mc > kMaxHalf)
        return fail(CFD_EINVAL, "cfd_scheme_create: size out of range");
    if (nc != nl) return fail(CFD_EINVAL, "cfd_scheme_create: closure rows must equal the implicit half-width");
    if (nc > 0 && !closure) return fail(CFD_EINVAL, "cfd_scheme_create: closure rows missing");
    if (std::fabs(lhs[nl] - 1.0) > 1e-15) return fail(CFD_EINVAL, "cfd_scheme_create: alpha^(d)_0 must be 1");
    Scheme s;
    s.d = d;
    s.order = order;
    s.nl = nl;
    s.m = m;
    s.nc = nc;
    s.mc = mc;
    for (int j = -nl; j <= nl; ++j) s.lhs[kMaxNL + j] = lhs[nl + j];
    for (int k = -m; k <= m; ++k) s.rhs[kMaxHalf + k] = rhs[m + k];
    for (int r = 0; r < nc; ++r)
        for (int k = -mc; k <= mc; ++k) s.cl[r][kMaxHalf + k] = closure[r * (2 * mc + 1) + mc + k];
    std::string err;
    cfd_status st = check_taylor(s, err);
    if (st == CFD_OK) st = check_centred(s, err);
    if (st == CFD_OK) st = check_symbol(s, err);
    if (st != CFD_OK) return fail(st, "cfd_scheme_create: " + err);
    s.name = "custom";
    *out = new cfd_scheme{s};
    return CFD_OK;
}

cfd_status cfd_scheme_get(const cfd_scheme *sc, int *d, int *order, int *nl, int *m, int *nc, int *mc,
                          double *lhs5, double *rhs11, double *closure22) {
    if (!sc) return fail(CFD_EINVAL, "cfd_scheme_get: null scheme");
    const Scheme &s = sc->s;
    if (d) *d = s.d;
    if (order) *order = s.order;
    if (nl) *nl = s.nl;
    if (m) *m = s.m;
    if (nc) *nc = s.nc;
    if (mc) *mc = s.mc;
    if (lhs5) std::memcpy(lhs5, s.lhs, sizeof s.lhs);
    if (rhs11) std::memcpy(rhs11, s.rhs, sizeof s.rhs);
    if (closure22) std::memcpy(closure22, s.cl, sizeof s.cl);
    return CFD_OK;
}

cfd_status cfd_scheme_design_biased(char family, int M, double lambda, int bias, cfd_scheme **out) {
    if (!out) return fail(CFD_EINVAL, "cfd_scheme_design_biased: null output");
    std::string err;
    Scheme s;
    cfd_status st = design_biased(family, M, lambda, bias, s, err);
    if (st != CFD_OK) return fail(st, err);
    *out = new cfd_scheme{s};
    return CFD_OK;
}

cfd_status cfd_scheme_dissipation(int r, double sigma, cfd_scheme **out) {
    if (!out) return fail(CFD_EINVAL, "cfd_scheme_dissipation: null output");
    std::string err;
    Scheme s;
    cfd_status st = design_dissipation(r, sigma, s, err);
    if (st != CFD_OK) return fail(st, err);
    *out = new cfd_scheme{s};
    return CFD_OK;
}

cfd_status cfd_scheme_get_biased(const cfd_scheme *sc, int *bias, int *order, double *alpha, double *a11,
                                 double *c12) {
    if (!sc) return fail(CFD_EINVAL, "cfd_scheme_get_biased: null scheme");
    const Scheme &s = sc->s;
    if (s.kind != 1) return fail(CFD_EINVAL, "cfd_scheme_get_biased: '" + s.name + "' is not a biased scheme");
    if (bias) *bias = s.bias;
    if (order) *order = s.order;
    if (alpha) *alpha = s.balpha;
    if (a11) std::memcpy(a11, s.ba, sizeof s.ba);
    if (c12) std::memcpy(c12, s.bc, sizeof s.bc);
    return CFD_OK;
}

cfd_status cfd_scheme_get_embedded(const cfd_scheme *sc, double *alpha2, int *m2) {
    if (!sc) return fail(CFD_EINVAL, "cfd_scheme_get_embedded: null scheme");
    const Scheme &s = sc->s;
    if (s.kind != 1) return fail(CFD_EINVAL, "cfd_scheme_get_embedded: '" + s.name + "' is not a biased scheme");
    if (alpha2) *alpha2 = s.ba2;
    if (m2) *m2 = s.emb;
    return CFD_OK;
}

cfd_status cfd_taylor_scheme(int dr, int L, int R, int nclass, const int *dI, const int *Lk, const int *Rk,
                             double *coef, int cap, int *order) {
    if (!coef || !order) return fail(CFD_EINVAL, "cfd_taylor_scheme: null output");
    std::vector<double> c;
    std::string err;
    int ord = 0;
    cfd_status st = taylor_scheme(dr, L, R, nclass, dI, Lk, Rk, c, ord, err);
    if (st != CFD_OK) return fail(st, err);
    if ((int)c.size() > cap) return fail(CFD_EINVAL, "cfd_taylor_scheme: coefficient array too small");
    std::memcpy(coef, c.data(), c.size() * sizeof(double));
    *order = ord;
    return CFD_OK;
}

cfd_status cfd_scheme_required_ghosts(const cfd_scheme *sc, cfd_boundary b, int *ng) {
    if (!sc || !ng) return fail(CFD_EINVAL, "cfd_scheme_required_ghosts: null argument");
    if (b != CFD_BOUNDARY_CLOSURE && b != CFD_BOUNDARY_PERIODIC)
        return fail(CFD_EINVAL, "cfd_scheme_required_ghosts: unknown boundary kind");
    *ng = required_ghosts(sc->s, b == CFD_BOUNDARY_PERIODIC);
    return CFD_OK;
}

void cfd_scheme_destroy(cfd_scheme *s) { delete s; }

cfd_status cfd_plan_create(const cfd_plan_desc *desc, cfd_plan **out) {
    if (!desc || !out) return fail(CFD_EINVAL, "cfd_plan_create: null argument");
    if (desc->nblocks < 1 || !desc->blocks) return fail(CFD_EINVAL, "cfd_plan_create: no blocks");
    if (desc->nfields < 1) return fail(CFD_EINVAL, "cfd_plan_create: nfields < 1");
    if (desc->nops < 1 || !desc->ops) return fail(CFD_EINVAL, "cfd_plan_create: no operators");
    if (desc->dtype != CFD_F64 && desc->dtype != CFD_F32 && desc->dtype != CFD_MIXED_BF16)
        return fail(CFD_EINVAL, "cfd_plan_create: unknown dtype");
    std::unique_ptr<cfd_plan> p(new cfd_plan);
    p->device = desc->device;
    p->dtype = desc->dtype;
    p->nfields = desc->nfields;
    p->blocks.assign(desc->blocks, desc->blocks + desc->nblocks);
    p->ops.assign(desc->ops, desc->ops + desc->nops);
    for (const cfd_op &op : p->ops) {
        if (!op.scheme) return fail(CFD_EINVAL, "cfd_plan_create: operator without scheme");
        if (op.dir < 0 || op.dir > 2) return fail(CFD_EINVAL, "cfd_plan_create: operator direction not in 0..2");
        if (op.field < -1 || op.field >= desc->nfields)
            return fail(CFD_EINVAL, "cfd_plan_create: operator field out of range");
        const Scheme &s = op.scheme->s;
        if (s.kind == 1 && s.bias == 0) {
            if (op.vel_field < 0 || op.vel_field >= desc->nfields)
                return fail(CFD_EINVAL, "cfd_plan_create: upwind operator '" + s.name +
                                            "' needs a velocity field index in 0..nfields-1");
        } else if (op.vel_field != -1) {
            return fail(CFD_EINVAL, "cfd_plan_create: vel_field must be -1 for operator '" + s.name +
                                        "' (only upwind pairs read a velocity field)");
        }
        if (s.kind == 1 && s.hermite) {
            if (op.aux_field < 0 || op.aux_field >= desc->nfields || op.field < 0)
                return fail(CFD_EINVAL, "cfd_plan_create: operator '" + s.name +
                                            "' samples f'': it needs one field and aux_field, the field holding "
                                            "its second derivative, in 0..nfields-1");
        } else if (op.aux_field != -1) {
            return fail(CFD_EINVAL, "cfd_plan_create: aux_field must be -1 for operator '" + s.name +
                                        "' (only U schemes read a sampled second derivative)");
        }
        if (s.kind == 1 && desc->dtype == CFD_MIXED_BF16)
            return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: biased schemes are not supported");
        if (op.dir2 != -1) {
            if (op.dir2 < 0 || op.dir2 > 2 || op.dir2 == op.dir)
                return fail(CFD_EINVAL, "cfd_plan_create: dir2 must be -1 or a direction other than dir");
            if (s.kind != 0 || s.d != 1 || scale_power(s) != 1)
                return fail(CFD_EINVAL, "cfd_plan_create: a mixed derivative needs a centred first-degree scheme, not '" +
                                            s.name + "'");
            if (desc->dtype == CFD_MIXED_BF16)
                return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: mixed derivatives are not supported");
        }
        p->schemes.push_back(s);
    }
    p->emb_sch.assign(p->ops.size(), -1);
    for (size_t o = 0; o < p->ops.size(); ++o) {
        const Scheme &s = p->schemes[o];
        if (s.kind != 1 || s.emb == 0) continue;
        Scheme e2;
        std::string err;
        char nm[16];
        std::snprintf(nm, sizeof nm, "(2)P1_%d", s.emb);
        cfd_status est = scheme_from_name(nm, e2, err);
        if (est != CFD_OK) return fail(est, "cfd_plan_create: embedded second derivative: " + err);
        p->emb_sch[o] = (int)p->schemes.size();
        p->schemes.push_back(e2);
    }
    int64_t slot = 0;
    for (const cfd_op &op : p->ops) {
        int nf = op.field < 0 ? desc->nfields : 1;
        p->op_nf.push_back(nf);
        p->op_slot.push_back(slot);
        slot += nf;
    }
    // validate blocks, resolve offsets
    int64_t in_cur = 0, out_cur = 0;
    for (size_t b = 0; b < p->blocks.size(); ++b) {
        const cfd_block &bl = p->blocks[b];
        for (int d = 0; d < 3; ++d) {
            if (bl.n[d] < 1) return fail(CFD_ESHAPE, "cfd_plan_create: block extent < 1");
            if (!(bl.h[d] > 0)) return fail(CFD_EINVAL, "cfd_plan_create: grid spacing must be positive");
            if (bl.boundary[d] != CFD_BOUNDARY_CLOSURE && bl.boundary[d] != CFD_BOUNDARY_PERIODIC)
                return fail(CFD_EINVAL, "cfd_plan_create: unknown boundary kind");
        }
        if (bl.ng < 0) return fail(CFD_EINVAL, "cfd_plan_create: negative ghost width");
        const int64_t ng = bl.ng;
        const int64_t in_n = (int64_t)desc->nfields * (bl.n[0] + 2 * ng) * (bl.n[1] + 2 * ng) * (bl.n[2] + 2 * ng);
        const int64_t out_n = slot * (int64_t)bl.n[0] * bl.n[1] * bl.n[2];
        if ((bl.in_offset < 0) != (bl.out_offset < 0))
            return fail(CFD_EINVAL, "cfd_plan_create: give both offsets of a block or neither");
        int64_t io = bl.in_offset < 0 ? in_cur : bl.in_offset;
        int64_t oo = bl.out_offset < 0 ? out_cur : bl.out_offset;
        p->in_off.push_back(io);
        p->out_off.push_back(oo);
        in_cur = std::max(in_cur, io + in_n);
        out_cur = std::max(out_cur, oo + out_n);
        for (size_t oo = 0; oo < 2 * p->ops.size(); ++oo) {
            const size_t o = oo / 2;
            if ((oo & 1) && p->ops[o].dir2 < 0) continue;   // second direction of a mixed derivative
            const Scheme &s = p->schemes[o];
            const int d = (oo & 1) ? p->ops[o].dir2 : p->ops[o].dir;
            const int per = bl.boundary[d] == CFD_BOUNDARY_PERIODIC;
            const int need = required_ghosts(s, per);
            if (bl.ng < need) {
                char buf[200];
                std::snprintf(buf, sizeof buf,
                              "block %zu: scheme '%s' needs %d ghost layers along direction %d, block has %d", b,
                              s.name.c_str(), need, d, bl.ng);
                return fail(CFD_EGHOST, buf);
            }
            const int N = bl.n[d];
            if (s.kind == 1) {
                if (N < 2) return fail(CFD_ESHAPE, "biased operator: lines need at least 2 nodes");
                continue;
            }
            if (!per && s.nl > 0 && N < 2 * s.nc + 1) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "block %zu: %d nodes along direction %d, closure needs >= %d", b, N,
                              d, 2 * s.nc + 1);
                return fail(CFD_ESHAPE, buf);
            }
            if (per && N < std::max(2 * s.nl + 1, std::max(s.m, s.mc))) {
                return fail(CFD_ESHAPE, "periodic line shorter than the stencil");
            }
            if (desc->dtype == CFD_MIXED_BF16) {
                if (!per)
                    return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: periodic lines only");
                if (N % 32 || N < 32 || N > 256)
                    return fail(CFD_EUNSUPPORTED, "mixed-precision dense path: line length must be 32..256, "
                                                  "a multiple of 32");
            }
        }
    }
    p->in_elems = in_cur;
    p->out_elems = out_cur;
    if (in_cur > (int64_t(1) << 40) || out_cur > (int64_t(1) << 40))
        return fail(CFD_EINVAL, "cfd_plan_create: layout too large");

    // passes: per block and direction, group operators by field selection and
    // fuse an odd-degree with an even-degree operator of equal band
    for (size_t b = 0; b < p->blocks.size(); ++b) {
        const cfd_block &bl = p->blocks[b];
        for (int d = 0; d < 3; ++d) {
            std::vector<int> ops_d;
            for (size_t o = 0; o < p->ops.size(); ++o)
                if (p->ops[o].dir == d && p->schemes[o].kind == 0 && p->ops[o].dir2 < 0) ops_d.push_back((int)o);
            std::vector<bool> used(p->ops.size(), false);
            for (int o : ops_d) {
                if (used[o]) continue;
                used[o] = true;
                PassHost ps;
                ps.block = (int)b;
                ps.dir = d;
                ps.field0 = p->ops[o].field < 0 ? 0 : p->ops[o].field;
                ps.nfield = p->ops[o].field < 0 ? p->nfields : 1;
                ps.N = bl.n[d];
                ps.ng = bl.ng;
                ps.periodic = bl.boundary[d] == CFD_BOUNDARY_PERIODIC;
                const Scheme &s0 = p->schemes[o];
                ps.nl = s0.nl;
                ps.nops = 1;
                ps.op[0] = o;
                ps.sch[0] = o;
                int partner = -1;
                for (int o2 : ops_d) {
                    if (desc->dtype == CFD_MIXED_BF16) break;   // the dense path runs one operator per pass
                    if (used[o2] || p->ops[o2].field != p->ops[o].field) continue;
                    const Scheme &s1 = p->schemes[o2];
                    if (s1.nl != s0.nl || s0.nl == 0 || (s0.d % 2) == (s1.d % 2)) continue;
                    // fuse only where a two-operator kernel class is compiled
                    const bool per = bl.boundary[d] == CFD_BOUNDARY_PERIODIC;
                    const int mi2 = std::max(s0.m, s1.m);
                    const int hw2 = std::max(std::max(s0.m, per ? 0 : s0.mc), std::max(s1.m, per ? 0 : s1.mc));
                    int Ls[16];
                    if (line_class_Ls(desc->dtype != CFD_F64, s0.nl, 2, 1, mi2, hw2, Ls, 16) == 0) continue;
                    partner = o2;
                    break;
                }
                if (partner >= 0) {
                    used[partner] = true;
                    ps.nops = 2;
                    int odd = (s0.d % 2) ? o : partner, even = (s0.d % 2) ? partner : o;
                    ps.op[0] = odd;
                    ps.sch[0] = odd;
                    ps.op[1] = even;
                    ps.sch[1] = even;
                    ps.par = 1;
                } else {
                    ps.par = (s0.d % 2) ? 1 : 0;
                }
                ps.mi = 0;
                ps.hw = 0;
                for (int k = 0; k < ps.nops; ++k) {
                    const Scheme &s = p->schemes[ps.sch[k]];
                    ps.mi = std::max(ps.mi, s.m);
                    ps.hw = std::max(ps.hw, std::max(s.m, ps.periodic ? 0 : s.mc));
                }
                p->passes.push_back(ps);
            }
        }
    }
    // the fused wave stage runs the wave operators' passes once more, in two
    // launches, with stage epilogues instead of stores
    if ((desc->dtype == CFD_F64 || desc->dtype == CFD_F32) && is_wave_plan(p.get())) {
        const size_t n = p->passes.size();
        for (size_t i = 0; i < n; ++i) {
            PassHost ps = p->passes[i];
            ps.ext = 2;
            ps.iomode = (ps.op[0] == 2 || ps.op[0] == 5) ? 4 : 3;
            p->passes.push_back(ps);
        }
        p->wave_fused = true;
    }
    // symmetrised mixed derivatives: the order with inner direction dj and
    // outer di needs D_dj f on the block extended by its ghost layers along di
    // (none if di is periodic).  One first-stage pass D_dj f -> scratch S_dj per
    // (block, fields, dj, scheme) covers every operator of the plan that needs
    // it: S_dj is extended along each outer direction those operators pair with
    // dj (the lines along dj through both extensions also run, unused).  For
    // each order a second-stage pass D_di S_dj -> scratch T over the interior;
    // the combine averages the two T.
    {
        int64_t scr = 0;
        struct Inner {
            int ext = 0;         // bit k: extended along k
            int64_t S0 = 0;      // scratch offset
            int64_t e[3] = {0, 0, 0};
        };
        for (size_t b = 0; b < p->blocks.size(); ++b) {
            const cfd_block &bl = p->blocks[b];
            const int64_t ng = bl.ng;
            const int64_t n[3] = {bl.n[0], bl.n[1], bl.n[2]};
            const int64_t PX = n[0] + 2 * ng, PY = n[1] + 2 * ng, PZ = n[2] + 2 * ng;
            const int64_t s_in[3] = {1, PX, PX * PY};
            const int64_t s_int[3] = {1, n[0], n[0] * n[1]};
            const int64_t npts = n[0] * n[1] * n[2];
            int64_t g[3];
            for (int k = 0; k < 3; ++k) g[k] = bl.boundary[k] == CFD_BOUNDARY_PERIODIC ? 0 : ng;
            // (scheme, first field, fields, inner direction) -> its scratch
            std::map<std::tuple<const void *, int, int, int>, Inner> inner;
            auto key_of = [&](const cfd_op &op, int dj) {
                const int nf = op.field < 0 ? p->nfields : 1, f0 = op.field < 0 ? 0 : op.field;
                return std::make_tuple((const void *)op.scheme, f0, nf, dj);
            };
            for (size_t o = 0; o < p->ops.size(); ++o) {
                const cfd_op &op = p->ops[o];
                if (op.dir2 < 0) continue;
                inner[key_of(op, op.dir2)].ext |= 1 << op.dir;
                inner[key_of(op, op.dir)].ext |= 1 << op.dir2;
            }
            for (auto &kv : inner) {
                const int f0 = std::get<1>(kv.first), nf = std::get<2>(kv.first), dj = std::get<3>(kv.first);
                Inner &in = kv.second;
                int64_t off = 0;
                for (int k = 0; k < 3; ++k) {
                    const int64_t gk = (in.ext >> k & 1) ? g[k] : 0;
                    in.e[k] = n[k] + 2 * gk;
                    off += gk * s_in[k];
                }
                const int64_t ss[3] = {1, in.e[0], in.e[0] * in.e[1]};
                in.S0 = scr;
                scr += nf * in.e[0] * in.e[1] * in.e[2];
                int o = -1;   // an operator of this group: scheme and output bookkeeping
                for (size_t q = 0; q < p->ops.size() && o < 0; ++q)
                    if (p->ops[q].dir2 >= 0 && (key_of(p->ops[q], p->ops[q].dir2) == kv.first ||
                                                key_of(p->ops[q], p->ops[q].dir) == kv.first))
                        o = (int)q;
                const Scheme &s = p->schemes[o];
                const int u = (dj == 0) ? 1 : 0, v = (dj == 2) ? 1 : 2;
                const bool per = bl.boundary[dj] == CFD_BOUNDARY_PERIODIC;
                PassHost ps;
                ps.block = (int)b;
                ps.dir = dj;
                ps.field0 = f0;
                ps.nfield = nf;
                ps.N = (int)n[dj];
                ps.ng = bl.ng;
                ps.periodic = per;
                ps.nl = s.nl;
                ps.nops = 1;
                ps.op[0] = ps.sch[0] = o;
                ps.par = 1;
                ps.mi = s.m;
                ps.hw = std::max(s.m, per ? 0 : s.mc);
                ps.iomode = 1;
                ps.custom = true;
                PassDesc &q = ps.geom;
                std::memset(&q, 0, sizeof q);
                q.in_base = p->in_off[b] + ng * (s_in[0] + s_in[1] + s_in[2]) - off;
                q.in_fstride = PX * PY * PZ;
                q.su = (int32_t)s_in[u];
                q.sv = (int32_t)s_in[v];
                q.sd = (int32_t)s_in[dj];
                q.out_base[0] = in.S0;
                q.out_fstride = in.e[0] * in.e[1] * in.e[2];
                q.osu = (int32_t)ss[u];
                q.osv = (int32_t)ss[v];
                q.osd = (int32_t)ss[dj];
                q.nu = (int32_t)in.e[u];
                q.nlines = (int32_t)(in.e[u] * in.e[v]);
                q.field0 = f0;
                q.N = ps.N;
                q.ng = ps.ng;
                q.periodic = per;
                q.nfield_pass = nf;
                p->passes.push_back(ps);
            }
            for (size_t o = 0; o < p->ops.size(); ++o) {
                const cfd_op &op = p->ops[o];
                if (op.dir2 < 0) continue;
                const Scheme &s = p->schemes[o];
                const int nf = op.field < 0 ? p->nfields : 1;
                const int64_t oo = p->out_off[b] + p->op_slot[o] * npts;
                for (int ord = 0; ord < 2; ++ord) {
                    const int dj = ord == 0 ? op.dir2 : op.dir;   // inner derivative
                    const int di = ord == 0 ? op.dir : op.dir2;   // outer derivative
                    const Inner &in = inner.at(key_of(op, dj));
                    const int64_t ss[3] = {1, in.e[0], in.e[0] * in.e[1]};
                    // lines along di over the interior of S_dj; its g[di] ghost layers along di
                    int64_t base = in.S0;
                    for (int k = 0; k < 3; ++k)
                        if (in.ext >> k & 1) base += g[k] * ss[k];
                    const int u = (di == 0) ? 1 : 0, v = (di == 2) ? 1 : 2;
                    const bool per = bl.boundary[di] == CFD_BOUNDARY_PERIODIC;
                    PassHost ps;
                    ps.block = (int)b;
                    ps.dir = di;
                    ps.field0 = op.field < 0 ? 0 : op.field;
                    ps.nfield = nf;
                    ps.N = (int)n[di];
                    ps.ng = (int)g[di];
                    ps.periodic = per;
                    ps.nl = s.nl;
                    ps.nops = 1;
                    ps.op[0] = ps.sch[0] = (int)o;
                    ps.par = 1;
                    ps.mi = s.m;
                    ps.hw = std::max(s.m, per ? 0 : s.mc);
                    // half of each order: the first stores it, the second adds its own
                    ps.iomode = ord == 0 ? 5 : 6;
                    ps.ext = ord == 0 ? 0 : 3;
                    ps.hscale = 0.5;
                    ps.custom = true;
                    PassDesc &q = ps.geom;
                    std::memset(&q, 0, sizeof q);
                    q.in_base = base;
                    q.in_fstride = in.e[0] * in.e[1] * in.e[2];
                    q.su = (int32_t)ss[u];
                    q.sv = (int32_t)ss[v];
                    q.sd = (int32_t)ss[di];
                    q.out_base[0] = oo;
                    q.out_fstride = npts;
                    q.osu = (int32_t)s_int[u];
                    q.osv = (int32_t)s_int[v];
                    q.osd = (int32_t)s_int[di];
                    q.nu = (int32_t)n[u];
                    q.nlines = (int32_t)(n[u] * n[v]);
                    q.field0 = 0;
                    q.N = ps.N;
                    q.ng = ps.ng;
                    q.periodic = per;
                    q.nfield_pass = nf;
                    p->passes.push_back(ps);
                }
                ++p->n_mixed;
            }
        }
        // W operators: their embedded (2)P1_M along the operator's direction over
        // the block interior, into scratch (lines through the interior only)
        for (size_t b = 0; b < p->blocks.size(); ++b) {
            const cfd_block &bl = p->blocks[b];
            const int64_t ng = bl.ng;
            const int64_t n[3] = {bl.n[0], bl.n[1], bl.n[2]};
            const int64_t PX = n[0] + 2 * ng, PY = n[1] + 2 * ng, PZ = n[2] + 2 * ng;
            const int64_t s_in[3] = {1, PX, PX * PY};
            const int64_t s_int[3] = {1, n[0], n[0] * n[1]};
            const int64_t npts = n[0] * n[1] * n[2];
            for (size_t o = 0; o < p->ops.size(); ++o) {
                if (p->emb_sch[o] < 0) continue;
                const cfd_op &op = p->ops[o];
                const Scheme &e2 = p->schemes[p->emb_sch[o]];
                const int nf = op.field < 0 ? p->nfields : 1, f0 = op.field < 0 ? 0 : op.field;
                const int ld = op.dir;
                const int u = (ld == 0) ? 1 : 0, v = (ld == 2) ? 1 : 2;
                const bool per = bl.boundary[ld] == CFD_BOUNDARY_PERIODIC;
                if (!per && n[ld] < 3)
                    return fail(CFD_ESHAPE, "W operator: closure lines need at least 3 nodes for the embedded "
                                            "second derivative");
                if (per && n[ld] < std::max(2 * e2.nl + 1, std::max(e2.m, e2.mc)))
                    return fail(CFD_ESHAPE, "W operator: periodic line shorter than the embedded stencil");
                const int64_t S0 = scr;
                scr += nf * npts;
                p->emb_off[std::make_pair((int)b, (int)o)] = S0;
                PassHost ps;
                ps.block = (int)b;
                ps.dir = ld;
                ps.field0 = f0;
                ps.nfield = nf;
                ps.N = (int)n[ld];
                ps.ng = bl.ng;
                ps.periodic = per;
                ps.nl = e2.nl;
                ps.nops = 1;
                ps.op[0] = (int)o;
                ps.sch[0] = p->emb_sch[o];
                ps.par = 0;
                ps.mi = e2.m;
                ps.hw = std::max(e2.m, per ? 0 : e2.mc);
                ps.iomode = 1;
                ps.custom = true;
                PassDesc &q = ps.geom;
                std::memset(&q, 0, sizeof q);
                q.in_base = p->in_off[b] + ng * (s_in[0] + s_in[1] + s_in[2]);
                q.in_fstride = PX * PY * PZ;
                q.su = (int32_t)s_in[u];
                q.sv = (int32_t)s_in[v];
                q.sd = (int32_t)s_in[ld];
                q.out_base[0] = S0;
                q.out_fstride = npts;
                q.osu = (int32_t)s_int[u];
                q.osv = (int32_t)s_int[v];
                q.osd = (int32_t)s_int[ld];
                q.nu = (int32_t)n[u];
                q.nlines = (int32_t)(n[u] * n[v]);
                q.field0 = f0;
                q.N = ps.N;
                q.ng = ps.ng;
                q.periodic = per;
                q.nfield_pass = nf;
                p->passes.push_back(ps);
            }
        }
        p->mscr_elems = scr;
    }
    // the descriptor is valid; from here on the device is needed
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(CFD_EDEVICE, "cfd_plan_create: no HIP device");
    }
    if (desc->device < 0 || desc->device >= ndev) return fail(CFD_EINVAL, "cfd_plan_create: bad device ordinal");
    HIPCHK(hipSetDevice(p->device));
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
            p->cus = prop.multiProcessorCount;
            p->max_lds = prop.sharedMemPerBlock;
        }
        (void)hipGetLastError();
    }
    p->xcd_interleave_ok = xcd_dispatch_ok(p->device);
    cfd_status st = upload_layout(p.get());
    if (st == CFD_OK && p->mscr_elems > 0) {
        const size_t es = elem_size(p->dtype);
        if (dmalloc(&p->d_mscr.p, (size_t)p->mscr_elems * es) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(CFD_ENOMEM, "cfd_plan_create: allocating the plan scratch");
        }
    }
    if (st == CFD_OK && dmalloc(&p->d_count.p, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(CFD_ENOMEM, "cfd_plan_create: allocating the result counter");
    }
    if (st == CFD_OK) st = build_biased(p.get());
    if (st == CFD_OK) st = build(p.get());
    if (st != CFD_OK) {
        p->release();
        return st;
    }
    *out = p.release();
    return CFD_OK;
}

cfd_status cfd_plan_sizes(const cfd_plan *p, long long *in_elems, long long *out_elems) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_sizes: null plan");
    if (in_elems) *in_elems = p->in_elems;
    if (out_elems) *out_elems = p->out_elems;
    return CFD_OK;
}

cfd_status cfd_plan_offsets(const cfd_plan *p, long long *in_offsets, long long *out_offsets) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_offsets: null plan");
    for (size_t b = 0; b < p->blocks.size(); ++b) {
        if (in_offsets) in_offsets[b] = p->in_off[b];
        if (out_offsets) out_offsets[b] = p->out_off[b];
    }
    return CFD_OK;
}

cfd_status cfd_plan_stats(const cfd_plan *p, int *launches, long long *items) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_stats: null plan");
    if (launches) {
        int n = 0;
        for (const Group &g : p->groups) n += !fused_iomode(g.iomode);
        *launches = n;
    }
    if (items) {
        long long n = 0;
        for (const Group &g : p->groups)
            if (!fused_iomode(g.iomode)) n += g.nitems;
        *items = n;
    }
    return CFD_OK;
}

cfd_status cfd_apply(cfd_plan *p, const void *in_dev, void *out_dev, void *stream) {
    if (!p || !in_dev || !out_dev) return fail(CFD_EINVAL, "cfd_apply: null argument");
    if (((uintptr_t)in_dev % 16) || ((uintptr_t)out_dev % 16))
        return fail(CFD_EINVAL, "cfd_apply: buffers must be 16-byte aligned");
    HIPCHK(hipSetDevice(p->device));
    return enqueue(p, in_dev, out_dev, (hipStream_t)stream);
}

cfd_status cfd_plan_capture_graph(cfd_plan *p, const void *in_dev, void *out_dev, void *stream) {
    (void)stream;
    if (!p || !in_dev || !out_dev) return fail(CFD_EINVAL, "cfd_plan_capture_graph: null argument");
    if (((uintptr_t)in_dev % 16) || ((uintptr_t)out_dev % 16))
        return fail(CFD_EINVAL, "cfd_plan_capture_graph: buffers must be 16-byte aligned");
    HIPCHK(hipSetDevice(p->device));
    p->drop_graph();
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    // Fallback: where the runtime cannot capture or instantiate the apply (or
    // the test hook says so), remember the buffers and replay it eagerly.
    auto fall_back = [&]() {
        (void)hipGetLastError();
        p->drop_graph();
        p->eager_in = in_dev;
        p->eager_out = out_dev;
        return CFD_OK;
    };
    if (g_fail_capture.exchange(false)) return fall_back();
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return fall_back();
    cfd_status st = enqueue(p, in_dev, out_dev, p->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != CFD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fall_back();
    p->graph = g;
    e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return fall_back();
    return CFD_OK;
}

cfd_status cfd_plan_launch_graph(cfd_plan *p, void *stream) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_launch_graph: null plan");
    HIPCHK(hipSetDevice(p->device));
    if (!p->gexec) {
        if (p->eager_in) return enqueue(p, p->eager_in, p->eager_out, (hipStream_t)stream);
        return fail(CFD_EINVAL, "cfd_plan_launch_graph: no graph captured");
    }
    HIPCHK(hipGraphLaunch(p->gexec, (hipStream_t)stream));
    return CFD_OK;
}

cfd_status cfd_plan_graph_status(const cfd_plan *p, int *status) {
    if (!p || !status) return fail(CFD_EINVAL, "cfd_plan_graph_status: null argument");
    *status = p->gexec ? 1 : (p->eager_in ? 2 : 0);
    return CFD_OK;
}

cfd_status cfd_plan_count_nonfinite(cfd_plan *p, const void *out_dev, void *stream, long long *count) {
    if (!p || !out_dev || !count) return fail(CFD_EINVAL, "cfd_plan_count_nonfinite: null argument");
    HIPCHK(hipSetDevice(p->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(p->d_count.p, 0, sizeof(unsigned long long), st));
    HIPCHK(launch_count_nonfinite(p->dtype != CFD_F64, p->out_elems, out_dev, (unsigned long long *)p->d_count.p, st));
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, p->d_count.p, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *count = (long long)c;
    return CFD_OK;
}

cfd_status cfd_plan_set_schedule(cfd_plan *p, int N, int xlines, int partitions, int flags) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_set_schedule: null plan");
    if (flags & ~(CFD_SCHED_PERSISTENT | CFD_SCHED_SPLIT_X | CFD_SCHED_XCD | CFD_SCHED_CONCURRENT))
        return fail(CFD_EINVAL, "cfd_plan_set_schedule: unknown flag");
    if (p->dtype == CFD_MIXED_BF16 && N > 0)
        return fail(CFD_EINVAL, "cfd_plan_set_schedule: the dense path has no partition schedule");
    if (N > 0) {
        const auto key = std::make_pair(N, xlines ? 1 : 0);
        if (partitions > 0) {
            bool any = false;
            for (const PassHost &ps : p->passes) {
                if (ps.N != N || (ps.dir == 0) != (xlines != 0) || fused_pass(ps)) continue;
                std::vector<int> c = candidate_Ps(ps, p->dtype != CFD_F64, p->max_lds);
                if (std::find(c.begin(), c.end(), partitions) == c.end())
                    return fail(CFD_EINVAL, "cfd_plan_set_schedule: no compiled kernel for that partition count");
                any = true;
            }
            if (!any) return fail(CFD_EINVAL, "cfd_plan_set_schedule: no such lines in the plan");
            p->sched_P[key] = partitions;
        } else {
            p->sched_P.erase(key);
        }
    }
    if ((flags & CFD_SCHED_XCD) && !(flags & CFD_SCHED_PERSISTENT) && !p->xcd_interleave_ok && p->dtype != CFD_MIXED_BF16)
        return fail(CFD_EUNSUPPORTED, "cfd_plan_set_schedule: the XCD-interleaved per-item order needs workgroups "
                                      "dealt round-robin over 8 XCDs, which this device did not show");
    p->persistent = (flags & CFD_SCHED_PERSISTENT) != 0;
    p->split_x = (flags & CFD_SCHED_SPLIT_X) != 0;
    p->xcd = (flags & CFD_SCHED_XCD) != 0;
    p->concurrent = (flags & CFD_SCHED_CONCURRENT) != 0;
    p->bconcurrent = p->concurrent;
    return build(p);
}

cfd_status cfd_plan_autotune(cfd_plan *p, const void *in_dev, void *out_dev, void *stream, const char *cache_path) {
    if (!p || !in_dev || !out_dev) return fail(CFD_EINVAL, "cfd_plan_autotune: null argument");
    HIPCHK(hipSetDevice(p->device));
    hipStream_t st = (hipStream_t)stream;
    std::string arch = "gfx";
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
        (void)hipGetLastError();
    }
    const bool f32 = p->dtype != CFD_F64;
    const char *dt = f32 ? "f32" : "f64";
    // the biased kernel classes' launches one after the other or on forked
    // streams, whichever makes the whole apply faster
    auto tune_biased = [&]() -> cfd_status {
        if (p->bgroups.size() < 2) return CFD_OK;
        hipEvent_t a0, a1;
        HIPCHK(hipEventCreate(&a0));
        HIPCHK(hipEventCreate(&a1));
        float best = 1e30f;
        bool bc = false;
        cfd_status r = CFD_OK;
        for (int conc = 0; conc <= 1 && r == CFD_OK; ++conc) {
            p->bconcurrent = conc;
            for (int w = 0; w < 3 && r == CFD_OK; ++w) r = enqueue(p, in_dev, out_dev, st);
            for (int trial = 0; trial < 3 && r == CFD_OK; ++trial) {
                (void)hipEventRecord(a0, st);
                for (int w = 0; w < 10 && r == CFD_OK; ++w) r = enqueue(p, in_dev, out_dev, st);
                (void)hipEventRecord(a1, st);
                (void)hipEventSynchronize(a1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, a0, a1);
                if (ms < best) {
                    best = ms;
                    bc = conc;
                }
            }
        }
        (void)hipEventDestroy(a0);
        (void)hipEventDestroy(a1);
        p->bconcurrent = bc;
        return r;
    };
    if (p->passes.empty()) {   // only biased operators: just that choice (reported as the plan's flag)
        cfd_status r = tune_biased();
        p->concurrent = p->bconcurrent;
        return r;
    }
    if (p->dtype == CFD_MIXED_BF16) {
        // only the grid kind: persistent or one workgroup per item
        hipEvent_t a0, a1;
        HIPCHK(hipEventCreate(&a0));
        HIPCHK(hipEventCreate(&a1));
        float best = 1e30f;
        bool bp = true;
        cfd_status r = CFD_OK;
        for (int pers = 1; pers >= 0 && r == CFD_OK; --pers) {
            p->persistent = pers;
            for (int w = 0; w < 2 && r == CFD_OK; ++w) r = enqueue(p, in_dev, out_dev, st);
            if (r != CFD_OK) break;
            (void)hipEventRecord(a0, st);
            for (int w = 0; w < 5 && r == CFD_OK; ++w) r = enqueue(p, in_dev, out_dev, st);
            (void)hipEventRecord(a1, st);
            (void)hipEventSynchronize(a1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, a0, a1);
            if (ms < best) { best = ms; bp = pers; }
        }
        (void)hipEventDestroy(a0);
        (void)hipEventDestroy(a1);
        p->persistent = bp;
        return r;
    }
    // one class per (line length, x or y/z, band, fused operators)
    std::map<std::tuple<int, int, int, int>, std::vector<int>> classes;
    for (const PassHost &ps : p->passes)
        if (!fused_pass(ps))
            classes[std::make_tuple(ps.N, ps.dir == 0 ? 1 : 0, ps.nl, ps.nops)] = candidate_Ps(ps, f32, p->max_lds);
    std::map<std::string, int> cache;
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string key;
        int v;
        while (f >> key >> v) cache[key] = v;
    }
    auto keyof = [&](const std::tuple<int, int, int, int> &k) {
        std::ostringstream s;
        s << "v5:" << arch << ":" << dt << ":N" << std::get<0>(k) << ":x" << std::get<1>(k) << ":nl" << std::get<2>(k)
          << ":ops" << std::get<3>(k);
        return s.str();
    };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // a candidate's time: the best of three runs of 10 applies after 3 warm-up
    // applies (single runs vary by several percent between candidates that
    // differ by less)
    auto time_apply = [&](float &ms) -> cfd_status {
        for (int w = 0; w < 3; ++w) {
            cfd_status s = enqueue(p, in_dev, out_dev, st);
            if (s != CFD_OK) return s;
        }
        const int reps = 10;
        ms = 1e30f;
        for (int trial = 0; trial < 3; ++trial) {
            HIPCHK(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) {
                cfd_status s = enqueue(p, in_dev, out_dev, st);
                if (s != CFD_OK) return s;
            }
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t / reps);
        }
        return CFD_OK;
    };
    // launch shape: persistent grid, XCD-aware queues or per-item grid (plain
    // or in XCD-interleaved order); x lines fused with y/z or split; launches
    // sequential or concurrent
    auto tune_shape = [&](float &best) -> cfd_status {
        best = 1e30f;
        int bmode = 1;
        bool bs = false, bc = false;
        cfd_status r = CFD_OK;
        // mode: 0 per-item grid, 1 persistent, 2 persistent with XCD queues,
        // 3 per-item grid in XCD-interleaved order
        for (int mode = 0; mode < 4 && r == CFD_OK; ++mode)
            for (int split = 0; split <= 1 && r == CFD_OK; ++split) {
                if (mode == 3 && !p->xcd_interleave_ok) break;
                for (int conc = 0; conc <= 1 && r == CFD_OK; ++conc) {
                    p->persistent = mode == 1 || mode == 2;
                    p->xcd = mode >= 2;
                    p->split_x = split;
                    p->concurrent = conc;
                    r = build(p);
                    int nplain = 0;
                    for (const Group &g : p->groups) nplain += !fused_iomode(g.iomode);
                    if (r == CFD_OK && conc && nplain < 2) continue;   // same as sequential
                    float ms = 0;
                    if (r == CFD_OK) r = time_apply(ms);
                    if (r == CFD_OK && ms < best) { best = ms; bmode = mode; bs = split; bc = conc; }
                }
            }
        p->persistent = bmode == 1 || bmode == 2;
        p->xcd = bmode >= 2;
        p->split_x = bs;
        p->concurrent = bc;
        return r;
    };
    // Partition presets: the default preference, and a compact one (the
    // fewest partitions with at most 16 rows for y/z lines and 12 for x
    // lines), under which every pass can use the kernel classes compiled
    // without long partitions (fewer registers, more waves per SIMD).  Tuning
    // one class at a time does not find the compact set: moving a single
    // class to another kernel adds a launch.
    auto apply_preset = [&](int which) {
        p->sched_P.clear();
        if (which == 0) return;
        for (const PassHost &ps : p->passes) {
            if (fused_pass(ps)) continue;
            int c[4];
            const int n = candidate_Ps(ps, f32, p->max_lds, c);
            const int cap = ps.dir == 0 ? 12 : 16;
            int pick = 0;
            for (int i = 0; i < n; ++i)
                if (partition_length(ps, f32, c[i]) <= cap && (!pick || c[i] < pick)) pick = c[i];
            if (pick) p->sched_P[std::make_pair(ps.N, ps.dir == 0 ? 1 : 0)] = pick;
        }
    };
    std::vector<std::string> new_lines;
    // 1. the launch shape under each preset; 2. partitions per class under the
    // best preset and shape; 3. the launch shape again with those partitions
    cfd_status result = CFD_OK;
    {
        float best = 1e30f;
        int bpre = 0;
        bool bpe = true, bx = false, bs = false, bc = false;
        for (int pre = 0; pre < 2 && result == CFD_OK; ++pre) {
            apply_preset(pre);
            float ms = 0;
            result = tune_shape(ms);
            if (result == CFD_OK && ms < best) {
                best = ms;
                bpre = pre;
                bpe = p->persistent;
                bx = p->xcd;
                bs = p->split_x;
                bc = p->concurrent;
            }
        }
        apply_preset(bpre);
        p->persistent = bpe;
        p->xcd = bx;
        p->split_x = bs;
        p->concurrent = bc;
    }
    const int shape = (p->persistent ? 1 : 0) | (p->split_x ? 2 : 0) | (p->xcd ? 4 : 0) | (p->concurrent ? 8 : 0);
    for (auto &kv : classes) {
        if (result != CFD_OK) break;
        const auto skey = std::make_pair(std::get<0>(kv.first), std::get<1>(kv.first));
        const std::string key = keyof(kv.first) + ":shape" + std::to_string(shape);
        auto hit = cache.find(key);
        if (hit != cache.end() && std::find(kv.second.begin(), kv.second.end(), hit->second) != kv.second.end()) {
            p->sched_P[skey] = hit->second;
            continue;
        }
        if (kv.second.size() < 2) continue;
        float best = 1e30f;
        int bestP = kv.second[0];
        for (int P : kv.second) {
            p->sched_P[skey] = P;
            result = build(p);
            if (result != CFD_OK) break;
            float ms;
            result = time_apply(ms);
            if (result != CFD_OK) break;
            if (ms < best) { best = ms; bestP = P; }
        }
        if (result != CFD_OK) break;
        p->sched_P[skey] = bestP;
        new_lines.push_back(key + " " + std::to_string(bestP));
    }
    if (result == CFD_OK) {
        float ms = 0;
        result = tune_shape(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != CFD_OK) return result;
    if (cache_path && !new_lines.empty()) {
        std::ofstream f(cache_path, std::ios::app);
        for (const std::string &l : new_lines) f << l << "\n";
    }
    result = build(p);
    // The winner must give bit for bit what the plain persistent grid gives
    // with the same partitions (the launch shape only decides which
    // workgroup runs which item); otherwise fall back to the plain shape.
    if (result == CFD_OK) {
        bool same = false;
        result = same_as_plain(p, in_dev, out_dev, st, same);
        if (result == CFD_OK && !same) {
            p->persistent = true;
            p->xcd = false;
            p->split_x = false;
            p->concurrent = false;
            result = build(p);
        }
    }
    if (result == CFD_OK) result = tune_biased();   // under the line kernels' schedule
    return result;
}

cfd_status cfd_plan_get_schedule(const cfd_plan *p, int *persistent, int *split_x, int *n_classes, int *N,
                                 int *xlines, int *partitions, int cap) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_get_schedule: null plan");
    if (persistent) *persistent = p->persistent ? (p->xcd ? 2 : 1) : 0;
    if (split_x) *split_x = p->split_x;
    std::map<std::pair<int, int>, int> used;
    for (const PassHost &ps : p->passes)
        if (!fused_pass(ps)) used[std::make_pair(ps.N, ps.dir == 0 ? 1 : 0)] = ps.P;
    if (n_classes) *n_classes = (int)used.size();
    int i = 0;
    for (auto &kv : used) {
        if (i >= cap) break;
        if (N) N[i] = kv.first.first;
        if (xlines) xlines[i] = kv.first.second;
        if (partitions) partitions[i] = kv.second;
        ++i;
    }
    return CFD_OK;
}

cfd_status cfd_plan_get_flags(const cfd_plan *p, int *flags) {
    if (!p || !flags) return fail(CFD_EINVAL, "cfd_plan_get_flags: null argument");
    *flags = (p->persistent ? CFD_SCHED_PERSISTENT : 0) | (p->split_x ? CFD_SCHED_SPLIT_X : 0) |
             (p->xcd ? CFD_SCHED_XCD : 0) | (p->concurrent ? CFD_SCHED_CONCURRENT : 0);
    return CFD_OK;
}

cfd_status cfd_halo_exchange(cfd_plan *p, void *data_dev, int bx, int by, int bz, void *stream) {
    if (!p || !data_dev) return fail(CFD_EINVAL, "cfd_halo_exchange: null argument");
    if (bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz != (int64_t)p->blocks.size())
        return fail(CFD_EINVAL, "cfd_halo_exchange: lattice does not match the plan's block count");
    const cfd_block &b0 = p->blocks[0];
    for (const cfd_block &b : p->blocks)
        if (b.n[0] != b0.n[0] || b.n[1] != b0.n[1] || b.n[2] != b0.n[2] || b.ng != b0.ng)
            return fail(CFD_EINVAL, "cfd_halo_exchange: blocks differ in shape");
    for (int d = 0; d < 3; ++d)
        if (b0.ng > b0.n[d]) return fail(CFD_ESHAPE, "cfd_halo_exchange: ghost width exceeds block extent");
    if (((uintptr_t)data_dev % elem_size(p->dtype))) return fail(CFD_EINVAL, "cfd_halo_exchange: misaligned buffer");
    {   // the kernel indexes within a field in 32 bits and puts the block-fields on the grid's y axis
        const int64_t g = b0.ng;
        const int64_t fe = (b0.n[0] + 2 * g) * (b0.n[1] + 2 * g) * (b0.n[2] + 2 * g);
        if (fe >= (int64_t(1) << 31) || (int64_t)p->nfields * bx * by * bz > 65535)
            return fail(CFD_EUNSUPPORTED, "cfd_halo_exchange: block or lattice too large");
    }
    HIPCHK(hipSetDevice(p->device));
    hipError_t e = launch_halo(p->dtype != CFD_F64, data_dev, (const int64_t *)p->d_inoff.p, b0.n[0], b0.n[1],
                               b0.n[2], b0.ng, p->nfields, bx, by, bz, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching halo exchange");
    return CFD_OK;
}

// Neighbour table of either sampling (shared = 1: vertex-centred blocks whose
// extremal nodes coincide with their neighbours').
static cfd_status set_neighbors_impl(cfd_plan *p, const int *nbr, int shared, const char *who) {
    if (!p || !nbr) return fail(CFD_EINVAL, std::string(who) + ": null argument");
    const int nb = (int)p->blocks.size();
    std::vector<int> pairs, vp[3];
    int64_t fmax = 0, vmax[3] = {0, 0, 0};
    char buf[240];
    for (int b = 0; b < nb; ++b)
        for (int face = 0; face < 6; ++face) {
            const int q = nbr[6 * b + face];
            if (q == -1) continue;
            if (q < 0 || q >= nb) return fail(CFD_EINVAL, std::string(who) + ": neighbour index out of range");
            const cfd_block &A = p->blocks[b], &B = p->blocks[q];
            const int d = face >> 1;
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;   // the directions along the face
            if (A.ng != B.ng || A.n[t0] != B.n[t0] || A.n[t1] != B.n[t1]) {
                std::snprintf(buf, sizeof buf, "%s: face %d of block %d does not conform to block %d (extents "
                              "along the face and ghost widths must agree)", who, face, b, q);
                return fail(CFD_ESHAPE, buf);
            }
            if (B.n[d] < A.ng + shared || (shared && A.n[d] < 2)) {
                std::snprintf(buf, sizeof buf, "%s: block %d has fewer than %d nodes along direction %d", who, q,
                              A.ng + shared, d);
                return fail(CFD_ESHAPE, buf);
            }
            if (shared && nbr[6 * q + (face ^ 1)] != b) {
                std::snprintf(buf, sizeof buf, "%s: vertex-centred faces must be mutual (block %d face %d names "
                              "block %d, whose opposite face does not name block %d)", who, b, face, q, b);
                return fail(CFD_EINVAL, buf);
            }
            const int64_t PX = A.n[0] + 2 * A.ng, PY = A.n[1] + 2 * A.ng, PZ = A.n[2] + 2 * A.ng;
            if (PX * PY * PZ * p->nfields >= (int64_t(1) << 40))
                return fail(CFD_EUNSUPPORTED, std::string(who) + ": block too large");
            fmax = std::max<int64_t>(fmax, (int64_t)A.ng * A.n[t0] * A.n[t1]);
            pairs.insert(pairs.end(), {b, face, q});
            if (shared && (face & 1)) {
                vp[d].insert(vp[d].end(), {b, q});
                vmax[d] = std::max<int64_t>(vmax[d], (int64_t)A.n[t0] * A.n[t1]);
            }
        }
    const int np = (int)(pairs.size() / 3);
    int64_t nslots = 0;
    for (int nf : p->op_nf) nslots += nf;
    nslots = std::max<int64_t>(nslots, p->nfields);
    bool big = fmax >= (int64_t(1) << 31) || (int64_t)np * p->nfields > 65535;
    for (int d = 0; d < 3; ++d) big = big || (int64_t)(vp[d].size() / 2) * nslots > 65535;
    if (big) return fail(CFD_EUNSUPPORTED, std::string(who) + ": faces or face-fields too many for one launch");
    HIPCHK(hipSetDevice(p->device));
    if (np > 0) HIPCHK(hipMemcpy(p->d_hpairs.p, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice));
    std::vector<int> allv;
    for (int d = 0; d < 3; ++d) {
        p->voff[d] = (int)(allv.size() / 2);
        p->nvp[d] = (int)(vp[d].size() / 2);
        p->vface_max[d] = (int)vmax[d];
        allv.insert(allv.end(), vp[d].begin(), vp[d].end());
    }
    if (!allv.empty()) HIPCHK(hipMemcpy(p->d_vpairs.p, allv.data(), allv.size() * sizeof(int), hipMemcpyHostToDevice));
    p->n_hpairs = np;
    p->hface_max = (int)fmax;
    p->hshift = shared;
    return CFD_OK;
}

cfd_status cfd_plan_set_neighbors(cfd_plan *p, const int *nbr) {
    return set_neighbors_impl(p, nbr, 0, "cfd_plan_set_neighbors");
}

cfd_status cfd_plan_set_neighbors_vc(cfd_plan *p, const int *nbr) {
    return set_neighbors_impl(p, nbr, 1, "cfd_plan_set_neighbors_vc");
}

cfd_status cfd_shared_node_average(cfd_plan *p, void *data_dev, int output, void *stream) {
    if (!p || !data_dev) return fail(CFD_EINVAL, "cfd_shared_node_average: null argument");
    if (p->n_hpairs < 0 || p->hshift != 1)
        return fail(CFD_EINVAL, "cfd_shared_node_average: no vertex-centred neighbour table set");
    if (((uintptr_t)data_dev % elem_size(p->dtype)))
        return fail(CFD_EINVAL, "cfd_shared_node_average: misaligned buffer");
    int nslots = p->nfields;
    if (output) {
        nslots = 0;
        for (int nf : p->op_nf) nslots += nf;
    }
    HIPCHK(hipSetDevice(p->device));
    const int64_t *off = (const int64_t *)(output ? p->d_outoff.p : p->d_inoff.p);
    for (int d = 0; d < 3; ++d) {
        hipError_t e = launch_shared_avg(p->dtype != CFD_F64, data_dev, off, (const int *)p->d_shapes.p,
                                         (const int *)p->d_vpairs.p + 2 * p->voff[d], p->nvp[d], nslots,
                                         output ? 0 : 1, d, p->vface_max[d], (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "launching the shared-node average");
    }
    return CFD_OK;
}

cfd_status cfd_halo_exchange_table(cfd_plan *p, void *data_dev, void *stream) {
    if (!p || !data_dev) return fail(CFD_EINVAL, "cfd_halo_exchange_table: null argument");
    if (p->n_hpairs < 0) return fail(CFD_EINVAL, "cfd_halo_exchange_table: no neighbour table set");
    if (((uintptr_t)data_dev % elem_size(p->dtype)))
        return fail(CFD_EINVAL, "cfd_halo_exchange_table: misaligned buffer");
    HIPCHK(hipSetDevice(p->device));
    hipError_t e = launch_halo_table(p->dtype != CFD_F64, data_dev, (const int64_t *)p->d_inoff.p,
                                     (const int *)p->d_shapes.p, (const int *)p->d_hpairs.p, p->n_hpairs, p->nfields,
                                     p->hface_max, p->hshift, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching the table ghost exchange");
    return CFD_OK;
}

cfd_status cfd_axpby(cfd_dtype dtype, long long n, double a, const void *x_dev, double b, void *y_dev,
                     void *stream) {
    if (n < 0 || (n > 0 && (!x_dev || !y_dev))) return fail(CFD_EINVAL, "cfd_axpby: bad argument");
    if (dtype != CFD_F64 && dtype != CFD_F32) return fail(CFD_EINVAL, "cfd_axpby: dtype must be F64 or F32");
    hipError_t e = launch_axpby(dtype == CFD_F32, n, a, x_dev, b, y_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching axpby");
    return CFD_OK;
}

cfd_status cfd_xpcy(cfd_dtype dtype, long long n, const void *x_dev, double c, const void *y_dev, void *z_dev,
                    void *stream) {
    if (n < 0 || (n > 0 && (!x_dev || !y_dev || !z_dev))) return fail(CFD_EINVAL, "cfd_xpcy: bad argument");
    if (dtype != CFD_F64 && dtype != CFD_F32) return fail(CFD_EINVAL, "cfd_xpcy: dtype must be F64 or F32");
    hipError_t e = launch_xpcy(dtype == CFD_F32, n, x_dev, c, y_dev, z_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching xpcy");
    return CFD_OK;
}

namespace {
cfd_status wave_stage(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev, const void *acc_in_dev,
                      void *acc_dev, const void *derivs_dev, double a, double b, int bx, int by, int bz, void *stream) {
    if (!p || !u0_dev || !src_dev || !acc_dev || !derivs_dev)
        return fail(CFD_EINVAL, "cfd_wave_rk_stage: null argument");
    // the plan must hold the five wave fields and the six first-derivative operators
    static const int want[6][2] = {{0, 1}, {1, 1}, {2, 1}, {0, 2}, {1, 3}, {2, 4}};
    if (p->nfields != 5 || p->ops.size() != 6)
        return fail(CFD_EINVAL, "cfd_wave_rk_stage: plan needs 5 fields and 6 operators");
    for (int o = 0; o < 6; ++o)
        if (p->ops[o].dir != want[o][0] || p->ops[o].field != want[o][1] || p->schemes[o].d != 1)
            return fail(CFD_EINVAL, "cfd_wave_rk_stage: operators must be D_x Pi, D_y Pi, D_z Pi, D_x psi_x, "
                                    "D_y psi_y, D_z psi_z (first derivatives)");
    if (p->dtype != CFD_F64 && p->dtype != CFD_F32) return fail(CFD_EINVAL, "cfd_wave_rk_stage: dtype");
    HIPCHK(hipSetDevice(p->device));
    const int nb = (int)p->blocks.size();
    if (p->nunits >= (int64_t(1) << 31)) return fail(CFD_EUNSUPPORTED, "cfd_wave_rk_stage: grid too large");
    const int64_t nunits64 = p->nunits;
    if (!acc_in_dev) acc_in_dev = acc_dev;
    const int *shapes = (const int *)p->d_shapes.p;
    hipError_t e = launch_wave_stage(p->dtype == CFD_F32, u0_dev, src_dev, stage_dev, acc_in_dev, acc_dev, derivs_dev,
                                     (const int64_t *)p->d_inoff.p, (const int64_t *)p->d_outoff.p, shapes,
                                     shapes + 4 * nb, nb, (int)nunits64, a, b, bx, by, bz, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching wave stage");
    return CFD_OK;
}
}  // namespace

cfd_status cfd_wave_rk_stage(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                             const void *acc_in_dev, void *acc_dev, const void *derivs_dev, double a, double b,
                             void *stream) {
    return wave_stage(p, u0_dev, src_dev, stage_dev, acc_in_dev, acc_dev, derivs_dev, a, b, 0, 0, 0, stream);
}

cfd_status cfd_wave_rk_stage_halo(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                                  const void *acc_in_dev, void *acc_dev, const void *derivs_dev, double a, double b,
                                  int bx, int by, int bz, void *stream) {
    if (!p) return fail(CFD_EINVAL, "cfd_wave_rk_stage_halo: null plan");
    if (bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz != (int64_t)p->blocks.size())
        return fail(CFD_EINVAL, "cfd_wave_rk_stage_halo: lattice does not match the plan's block count");
    const cfd_block &b0 = p->blocks[0];
    for (const cfd_block &bl : p->blocks)
        if (bl.n[0] != b0.n[0] || bl.n[1] != b0.n[1] || bl.n[2] != b0.n[2] || bl.ng != b0.ng)
            return fail(CFD_EINVAL, "cfd_wave_rk_stage_halo: blocks differ in shape");
    for (int d = 0; d < 3; ++d)
        if (b0.ng > b0.n[d]) return fail(CFD_ESHAPE, "cfd_wave_rk_stage_halo: ghost width exceeds block extent");
    return wave_stage(p, u0_dev, src_dev, stage_dev, acc_in_dev, acc_dev, derivs_dev, a, b, bx, by, bz, stream);
}

cfd_status cfd_wave_rk_stage_fused(cfd_plan *p, const void *u0_dev, const void *src_dev, void *stage_dev,
                                   const void *acc_in_dev, void *acc_dev, void *work_dev, double a, double b, int bx,
                                   int by, int bz, void *stream) {
    if (!p || !u0_dev || !src_dev || !acc_dev || !work_dev)
        return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: null argument");
    if (!is_wave_plan(p))
        return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: operators must be D_x Pi, D_y Pi, D_z Pi, D_x psi_x, "
                                "D_y psi_y, D_z psi_z (first derivatives) on 5 fields");
    if (!p->wave_fused)
        return fail(CFD_EUNSUPPORTED, "cfd_wave_rk_stage_fused: available for FP64 and FP32 plans only");
    if (p->iter_n > 0)
        return fail(CFD_EUNSUPPORTED, "cfd_wave_rk_stage_fused: not with the hybrid closure iteration");
    if (!p->wave_fused_ok)
        return fail(CFD_EUNSUPPORTED, "cfd_wave_rk_stage_fused: no fused kernel compiled for this scheme and line "
                                      "length");
    if (!acc_in_dev) acc_in_dev = acc_dev;
    if (stage_dev == src_dev || acc_dev == src_dev || (stage_dev && stage_dev == acc_dev) ||
        (stage_dev && stage_dev == u0_dev))
        return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: stage and acc must be buffers of their own (not src, "
                                "not each other; stage not u0)");
    if (work_dev == u0_dev || work_dev == src_dev || work_dev == stage_dev || work_dev == acc_in_dev ||
        work_dev == acc_dev)
        return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: work must be a buffer of its own");
    const bool lattice = bx != 0 || by != 0 || bz != 0;
    if (lattice) {
        if (bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz != (int64_t)p->blocks.size())
            return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: lattice does not match the plan's block count");
        const cfd_block &b0 = p->blocks[0];
        for (const cfd_block &bl : p->blocks)
            if (bl.n[0] != b0.n[0] || bl.n[1] != b0.n[1] || bl.n[2] != b0.n[2] || bl.ng != b0.ng)
                return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: blocks differ in shape");
        for (int d = 0; d < 3; ++d)
            if (b0.ng > b0.n[d]) return fail(CFD_ESHAPE, "cfd_wave_rk_stage_fused: ghost width exceeds block extent");
    }
    for (const void *q : {u0_dev, src_dev, (const void *)stage_dev, acc_in_dev, (const void *)acc_dev,
                          (const void *)work_dev})
        if ((uintptr_t)q % 16) return fail(CFD_EINVAL, "cfd_wave_rk_stage_fused: buffers must be 16-byte aligned");
    HIPCHK(hipSetDevice(p->device));
    RkArgs rk{};
    rk.u0 = u0_dev;
    rk.stage = stage_dev;
    rk.acc_in = acc_in_dev;
    rk.acc = acc_dev;
    rk.epi = (const EpiDesc *)p->d_epi.p;
    rk.in_off = (const int64_t *)p->d_inoff.p;
    rk.a = a;
    rk.b = b;
    rk.lat[0] = lattice ? bx : 0;
    rk.lat[1] = lattice ? by : 0;
    rk.lat[2] = lattice ? bz : 0;
    rk.acc_is_u0 = acc_in_dev == u0_dev;
    return enqueue_wave_fused(p, src_dev, work_dev, rk, (hipStream_t)stream);
}

cfd_status cfd_plan_set_iteration(cfd_plan *p, int iterations, int bx, int by, int bz) {
    if (!p) return fail(CFD_EINVAL, "cfd_plan_set_iteration: null plan");
    if (iterations < 0) return fail(CFD_EINVAL, "cfd_plan_set_iteration: negative iteration count");
    if (p->dtype == CFD_MIXED_BF16)
        return fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: not available on the dense mixed-precision path");
    if (iterations > 0 && p->n_mixed > 0)
        return fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: the plan holds mixed derivatives");
    if (iterations > 0 && !p->emb_off.empty())
        return fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: the plan holds W operators (their embedded second "
                                      "derivative has no iterated closure)");
    for (size_t o = 0; o < p->ops.size() && iterations > 0; ++o)
        if (p->schemes[o].kind == 1 && p->schemes[o].hermite)
            return fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: the plan holds U operators (sampled f'')");
    const int c = 2;
    auto restore = [&]() {
        p->release_biased_iteration();
        if (!p->base_schemes.empty()) p->schemes = p->base_schemes;
        p->base_schemes.clear();
        for (PassHost &ps : p->passes) ps.ext = fused_pass(ps) ? 2 : (ps.iomode == 6 ? 3 : 0);
        p->iter_n = 0;
    };
    if (iterations == 0) {
        restore();
        for (PassHost &ps : p->passes) {
            if (fused_pass(ps)) continue;   // never changed by the iteration
            ps.mi = ps.hw = 0;
            for (int k = 0; k < ps.nops; ++k) {
                const Scheme &s = p->schemes[ps.sch[k]];
                ps.mi = std::max(ps.mi, s.m);
                ps.hw = std::max(ps.hw, std::max(s.m, ps.periodic ? 0 : s.mc));
            }
        }
        HIPCHK(hipSetDevice(p->device));
        return build(p);
    }
    if (bx < 1 || by < 1 || bz < 1 || (int64_t)bx * by * bz != (int64_t)p->blocks.size())
        return fail(CFD_EINVAL, "cfd_plan_set_iteration: lattice does not match the plan's block count");
    const cfd_block &b0 = p->blocks[0];
    for (const cfd_block &b : p->blocks) {
        if (b.n[0] != b0.n[0] || b.n[1] != b0.n[1] || b.n[2] != b0.n[2] || b.ng != b0.ng)
            return fail(CFD_EINVAL, "cfd_plan_set_iteration: blocks differ in shape");
        for (int d = 0; d < 3; ++d)
            if (b.boundary[d] != CFD_BOUNDARY_CLOSURE)
                return fail(CFD_EINVAL, "cfd_plan_set_iteration: blocks must use the block closure in every "
                                        "direction (the lattice wraps)");
    }
    std::vector<Scheme> base = p->base_schemes.empty() ? p->schemes : p->base_schemes;
    std::vector<Scheme> it(base.size());
    for (size_t o = 0; o < base.size(); ++o) {
        if (base[o].kind == 1) {
            // biased (Eq. iter_left_X): the same scheme, every row interior and the
            // entering value k^c = k*_- - 1 (k*_+ + 1) from the neighbour; lines of at
            // most the partitioned kernel's length, and ghosts for the interior
            // stencil on the first and last rows
            it[o] = base[o];
            const int N = b0.n[p->ops[o].dir];
            if (N > kBiasMaxPN)
                return fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: iterated biased closures need lines of at most "
                                              "64 nodes");
            int la = 0, ra = 0;
            for (int m = -kBiasHalf; m <= kBiasHalf; ++m)
                if (base[o].ba[m + kBiasHalf] != 0) {
                    la = std::max(la, -m);
                    ra = std::max(ra, m);
                }
            const int need = std::max(required_ghosts(base[o], 0), std::max(la, ra));
            if (b0.ng < need) {
                char buf[200];
                std::snprintf(buf, sizeof buf, "cfd_plan_set_iteration: scheme '%s' iterated needs %d ghost layers, "
                              "blocks have %d", base[o].name.c_str(), need, b0.ng);
                return fail(CFD_EGHOST, buf);
            }
            continue;
        }
        std::string err;
        cfd_status st = make_iterated(base[o], c, it[o], err);
        if (st != CFD_OK) return fail(st, "cfd_plan_set_iteration: scheme '" + base[o].name + "': " + err);
        const int need = std::max(required_ghosts(base[o], 0), required_ghosts(it[o], 0));
        if (b0.ng < need) {
            char buf[200];
            std::snprintf(buf, sizeof buf, "cfd_plan_set_iteration: scheme '%s' iterated needs %d ghost layers, "
                          "blocks have %d", base[o].name.c_str(), need, b0.ng);
            return fail(CFD_EGHOST, buf);
        }
        if (b0.n[p->ops[o].dir] < 2 * c + 1)
            return fail(CFD_ESHAPE, "cfd_plan_set_iteration: block too short for the iteration's end nodes");
    }
    p->base_schemes = base;
    p->schemes = it;
    for (PassHost &ps : p->passes) {
        if (fused_pass(ps)) continue;   // the fused wave stage is off while iterating
        ps.ext = 1;
        ps.mi = ps.hw = 0;
        for (int k = 0; k < ps.nops; ++k) {
            const Scheme &s = p->schemes[ps.sch[k]];
            ps.mi = std::max(ps.mi, s.m);
            ps.hw = std::max(ps.hw, std::max(s.m, s.mc));
        }
    }
    p->iter_n = iterations;
    p->iter_c = c;
    p->lat[0] = bx;
    p->lat[1] = by;
    p->lat[2] = bz;
    HIPCHK(hipSetDevice(p->device));
    cfd_status st = build(p);
    if (st == CFD_OK && p->nbitems > 0) {
        // biased passes: end-value buffers and, per pass, the passes of its
        // neighbours along its lines on the periodic lattice
        p->release_biased_iteration();
        const size_t es = elem_size(p->dtype);
        const int nbops = (int)(p->bpinfo.size() / p->blocks.size());
        std::vector<int64_t> recs;
        int64_t emax = 0;
        for (size_t i = 0; i < p->bpinfo.size(); ++i) {
            const auto &bi = p->bpinfo[i];
            const int b = (int)bi[0], o = (int)bi[1], d = p->ops[o].dir;
            int k[3] = {b % bx, (b / bx) % by, b / (bx * by)};
            int km[3] = {k[0], k[1], k[2]}, kp[3] = {k[0], k[1], k[2]};
            km[d] = (k[d] + p->lat[d] - 1) % p->lat[d];
            kp[d] = (k[d] + 1) % p->lat[d];
            const int bm = (km[2] * by + km[1]) * bx + km[0], bp = (kp[2] * by + kp[1]) * bx + kp[0];
            const int slot = (int)(i % nbops);   // the same operator's pass in the neighbour
            recs.insert(recs.end(), {bi[2], p->bpinfo[(size_t)bm * nbops + slot][2],
                                     p->bpinfo[(size_t)bp * nbops + slot][2], bi[3]});
            emax = std::max(emax, bi[3]);
        }
        hipError_t e = dmalloc(&p->d_bev.p, (size_t)std::max<int64_t>(1, 2 * p->bev_entries) * es);
        if (e == hipSuccess) e = dmalloc(&p->d_bends.p, (size_t)std::max<int64_t>(1, 2 * p->bev_entries) * es);
        if (e == hipSuccess) e = dmalloc(&p->d_bgrecs.p, std::max<size_t>(1, recs.size()) * sizeof(int64_t));
        if (e == hipSuccess && !recs.empty())
            e = hipMemcpy(p->d_bgrecs.p, recs.data(), recs.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess || p->bpinfo.size() > 65535) {
            (void)hipGetLastError();
            st = e != hipSuccess ? hip_fail(e, "cfd_plan_set_iteration: biased end-value buffers")
                                 : fail(CFD_EUNSUPPORTED, "cfd_plan_set_iteration: more than 65535 biased passes");
        }
        p->bev_max = emax;
    }
    if (st != CFD_OK) {
        restore();
        (void)build(p);
    }
    return st;
}

void cfd_debug_fail_alloc(long long n) { g_alloc_fail_after.store(n < 0 ? -1 : n); }

void cfd_debug_fail_capture(int on) { g_fail_capture.store(on != 0); }

void cfd_plan_destroy(cfd_plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    p->release();
    delete p;
}

}  // extern "C"
