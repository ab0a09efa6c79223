// Line kernel of the MI355X compact finite-difference library (gfx950).
//
// Line operator (arXiv 2302.14858, Eq. sch_cent_om and its matrix form
// Eqs. diff_mat_subL / diff_mat_subR): on every grid line of N nodes the
// derivative f~ solves  D_L f~ = h^-d D_R f,  where D_L has identity rows on
// the block-closure rows and the banded alpha^(d) rows elsewhere, and D_R has
// the explicit closure stencil or the interior stencil alpha^(0).  Periodic
// lines use the circulant operator instead.
//
// GPU decomposition (not from the paper, whose TDMA runs one line at a time):
//  * a line is cut into P partitions of L = N/P consecutive rows; a workgroup
//    of 4 wavefronts holds 4/P groups of 64 lines, and each wavefront owns one
//    partition of one group: lane = line, so the line-independent tables a
//    wavefront reads are uniform (scalar loads);
//  * lines along y and z are read straight from HBM: consecutive lanes are
//    consecutive x, so every load and store is coalesced;
//  * lines along x are contiguous in memory: the workgroup first stages its
//    lines (with ghosts) in LDS with coalesced loads, the lanes read their line
//    from LDS, and the results go back through LDS to coalesced stores;
//  * each lane streams its partition once: the RHS stencil is evaluated from a
//    register ring and fused with forward elimination, then back substitution
//    gives the partition-local solution y;
//  * partitions are coupled through 2*nl boundary unknowns each.  Their values
//    follow from the boundary entries of every partition's y by one fixed
//    linear map (rows of the inverse reduced system): the lanes of a line
//    exchange those entries through LDS and correct
//    x = y - sum(boundary value * spike vector).  For periodic lines the same
//    algebra closes the wrap-around (the Woodbury form of the cyclic solve).
// All line-independent quantities are built once per plan in FP64 on the GPU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfd_internal.h"

namespace cfd {

constexpr int kXCD = 8;   // accelerator complex dies (each with its own L2)

// Wavefronts per workgroup: a class is compiled for WG = 4 (items of P = 1, 2
// or 4 partitions, 4 / P groups of 64 lines) or WG = 8 (items of P = 8
// partitions, one group of 64 lines).  x items share the exchange area with
// their tile: the exchange runs after every lane has read its inputs from the
// tile and before the results are staged back into it.

// Derivatives are written once and not read again by this launch: streaming
// (non-temporal) stores keep them from evicting the input lines that the other
// directions' passes over the same block-field re-read from L2.
#ifndef CFD_NT_STORES
#define CFD_NT_STORES 1
#endif
template <typename T>
__device__ __forceinline__ void store_out(T *p, T v) {
#if CFD_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Per-item context shared by the template bodies.
template <typename T>
struct LineCtx {
    const PassDesc *pd;
    const T *tb[2];         // tables of the operators
    const T *src;           // global: node 0 of this lane's line (non-x)
    T *tile;                // LDS tile of staged x-lines (x only)
    T *exch;                // LDS exchange area
    int P, p, sub, g;       // partitions, this wave's partition, line group, lane
    int tpitch;             // tile row pitch (elements)
    int trow;               // this lane's tile row
    int C, chunk;           // x lines: column chunks of the tile, this wave's chunk
    const T *fbase;         // x lines: node (0, 0, 0) of the item's field
    int line0;              // x lines: first line of the item
    bool periodic;
    T em[2], ep[2];         // iterated closures: this lane's end values per op
};

// One lane: the p-th partition (L rows) of its line, all NOPS operators.
// Leaves the solution (times h^-d) in y.
template <typename T, int NL, int NOPS, int PAR, int MI, int HW, int L, bool X, bool PAD, int XM>
__device__ __forceinline__ void solve_partition(const LineCtx<T> &c, T (&y)[NOPS][L], T (&fin)[L + 2 * HW]) {
    const PassDesc &pd = *c.pd;
    const int N = pd.N;
    const int ng = pd.ng;
    const int k0 = c.p * L;
    const int64_t sd = pd.sd;

    const int Npad = c.P * L;
    // node j of this line (global path) for the first and last partition,
    // whose halo can leave the line: out-of-block nodes read as 0 (their
    // weights are zero; a class compiled for a wider ring than the scheme
    // reaches, e.g. an explicit 6th-order stencil at ng = 3 in a class for
    // half-width 5, also meets nodes past the stored ghosts here)
    auto edge_load = [&](int j) -> T {
        if (c.periodic) {
            if (j < 0) j += N;
            if (j >= N) j -= N;
            return c.src[(int64_t)j * sd];
        }
        if (j < -ng || j >= N + ng) return T(0);
        return c.src[(int64_t)j * sd];
    };

    // every input node of the partition (its rows and a halo of HW on each
    // side) is requested before any arithmetic, so all of the partition's loads
    // are in flight together.  x lines: the caller has read fin from the tile.
    if constexpr (!X) {
        // only the first and last partition's halo can leave the stored line
        // (nodes -ng .. N+ng-1): an inner partition starts at k0 >= L >= HW,
        // and the host admits P partitions of a closure line only if
        // (P-1) L + HW <= N + ng (periodic lines wrap, and L >= HW)
        const bool lo_edge = c.p == 0;
        const bool hi_edge = c.p == c.P - 1;
        // walk a pointer along the line: one stride add per node keeps the
        // addresses in vector registers instead of one scalar offset per node
        const T *q = c.src + (int64_t)(k0 - HW) * sd;
#pragma unroll
        for (int t = 0; t < L + 2 * HW; ++t) {
            const int j = k0 - HW + t;
            const bool edge = (t < HW && lo_edge) || ((t >= L + HW || (PAD && t >= HW + L - (Npad - N))) && hi_edge);
            fin[t] = edge ? edge_load(j) : *q;
            q += sd;
        }
    }
    const bool first = (c.p == 0) && !c.periodic;
    // the last partition of a closure line: its last NL rows are the right
    // closure rows, unless the line is padded (PAD): then rows >= N are
    // decoupled identity rows with zero right-hand side and the closure rows
    // sit at runtime positions
    const bool last = (c.p == c.P - 1) && !c.periodic;

#pragma unroll
    for (int i = 0; i < L; ++i) {
        const T *f = fin + i;   // f[HW + m] is node k0 + i + m
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const T *cf = c.tb[o];
            T r;
            if ((PAR >> o) & 1) {   // antisymmetric interior stencil
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
                    const T *cl = cf + kCoefCL + i * 11;
                    T s = T(0);
#pragma unroll
                    for (int m = -HW; m <= HW; ++m) s += cl[5 + m] * f[HW + m];
                    r = s;
                }
                if constexpr (PAD) {
                    if (last) {
                        const int k = k0 + i;
                        if (k >= N - NL) {
                            if (k < N) {
                                const T *cr = cf + kCoefCR + (N - 1 - k) * 11;
                                T s = T(0);
#pragma unroll
                                for (int m = -HW; m <= HW; ++m) s += cr[5 + m] * f[HW + m];
                                r = s;
                            } else {
                                r = T(0);
                            }
                        }
                    }
                } else {
                    if (i >= L - NL && last) {
                        const T *cr = cf + kCoefCR + (L - 1 - i) * 11;
                        T s = T(0);
#pragma unroll
                        for (int m = -HW; m <= HW; ++m) s += cr[5 + m] * f[HW + m];
                        r = s;
                    }
                }
                // forward elimination with the partition-local factors
                const T *fw = cf + kCoefHdr + (int64_t)(k0 + i) * 2;
                if (i >= 1) r -= fw[0] * y[o][i - 1];
                if (NL >= 2 && i >= 2) r -= fw[1] * y[o][i - 2];
            }
            y[o][i] = r;
        }
    }

    if constexpr (NL > 0) {
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const T *cf = c.tb[o];
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                const T *bw = cf + kCoefHdr + (int64_t)Npad * 2 + (int64_t)(k0 + i) * 3;
                T v = y[o][i];
                if (i + 1 < L) v -= bw[0] * y[o][i + 1];
                if (NL >= 2 && i + 2 < L) v -= bw[1] * y[o][i + 2];
                y[o][i] = v * bw[2];
            }
        }
        if (c.periodic || c.P > 1) {
            const int B = 2 * NL * c.P;
            const int Bp = B | 1;
            // x lines: the exchange area overlays the tile, which other waves
            // may still be reading their inputs from
            if constexpr (X) __syncthreads();
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                T *row = c.exch + ((int64_t)(c.sub * NOPS + o) * 64 + c.g) * Bp + c.p * 2 * NL;
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    row[t] = y[o][t];
                    row[NL + t] = y[o][L - NL + t];
                }
            }
            __syncthreads();
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                const T *cf = c.tb[o];
                const T *spk = cf + kCoefHdr + (int64_t)Npad * 5 + (int64_t)c.p * 2 * NL * L;
                const T *krow = cf + kCoefHdr + (int64_t)Npad * 5 + (int64_t)c.P * 2 * NL * L + (int64_t)c.p * 2 * NL * B;
                const T *row = c.exch + ((int64_t)(c.sub * NOPS + o) * 64 + c.g) * Bp;
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
        }
    }
#pragma unroll
    for (int o = 0; o < NOPS; ++o) {
        const T hinv = (T)pd.hinv[o];
#pragma unroll
        for (int i = 0; i < L; ++i) y[o][i] *= hinv;
    }
    if constexpr (XM == 1) {
        // iterated closure (Eq. iter_center_P): the block system carries the
        // two end values on its closure rows; add their responses (the
        // influence vectors of the table, zero on padding rows)
        const int64_t B = 2 * NL * c.P;
#pragma unroll
        for (int o = 0; o < NOPS; ++o) {
            const T *gv = c.tb[o] + kCoefHdr + (int64_t)Npad * 5 + (int64_t)c.P * 2 * NL * L + (int64_t)c.P * 2 * NL * B;
#pragma unroll
            for (int i = 0; i < L; ++i) y[o][i] += c.em[o] * gv[k0 + i] + c.ep[o] * gv[Npad + k0 + i];
        }
    }
}

// Stage the x-lines of this item in LDS: column t of row r holds node n0 + t
// of line line0 + r, t < W (zero outside the ghosts, wrapped for periodic
// lines; rows past the last line read as zero).  Thread tid owns the node
// pair tid % CW (CW = W / 2 pairs per row) of the rows tid / CW + k * RPP,
// RPP = 256 / CW rows per pass: its line advances by RPP per pass without a
// division, and the loads of BATCH passes are in flight together before their
// LDS writes.  W is even (partition lengths and 2 HW are).
template <typename T, int HW, int WG>
__device__ __forceinline__ void stage_x(const PassDesc &pd, const T *base, int line0, int nrows, int n0, int W,
                                        T *tile, int tpitch, bool periodic) {
    constexpr int NT = 64 * WG;
    constexpr int BATCH = 8;
    const int N = pd.N, ng = pd.ng;
    const int CW = W >> 1;
    const int RPP = NT / CW;
    const int tid = threadIdx.x;
    const int r0 = tid / CW;
    const int c2 = tid - r0 * CW;
    if (r0 >= RPP) return;   // no barrier inside: idle threads may leave early
    // source offsets of the pair's two nodes within a line (-1: outside, reads 0)
    int j[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int jj = n0 + 2 * c2 + h;
        if (periodic) {
            if (jj < 0) jj += N;
            if (jj >= N) jj -= N;
        } else if (jj < -ng || jj >= N + ng) {
            jj = INT32_MIN;
        }
        j[h] = jj;
    }
    const int nr = min(nrows, pd.nlines - line0);   // rows that are real lines
    int line = line0 + r0;
    int lu = line % pd.nu, lv = line / pd.nu;
    for (int rb = r0; rb < nrows; rb += BATCH * RPP) {
        T v[BATCH][2];
        int dst[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int r = rb + b * RPP;
            dst[b] = r < nrows ? r * tpitch + 2 * c2 : -1;
            const T *row = base + (int64_t)lv * pd.sv + (int64_t)lu * pd.su;
#pragma unroll
            for (int h = 0; h < 2; ++h) v[b][h] = (r < nr && j[h] != INT32_MIN) ? row[j[h]] : T(0);
            lu += RPP;
            while (lu >= pd.nu) {
                lu -= pd.nu;
                ++lv;
            }
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
            if (dst[b] >= 0) {
                tile[dst[b]] = v[b][0];
                tile[dst[b] + 1] = v[b][1];
            }
    }
}

// Write the x results staged in the tile (row r = line line0 + r, pitch
// opitch, ncols columns) to the interior output rows of length N:
// consecutive x-lines of one field are consecutive rows of the output.
// Thread tid owns node pair tid % CO of rows tid / CO + k * RPP.
template <typename T, int WG, bool ACC = false>
__device__ __forceinline__ void store_x(T *dst, const T *tile, int nrows, int N, int ncols, int opitch) {
    constexpr int NT = 64 * WG;
    const int CO = (ncols + 1) >> 1;
    const int RPP = NT / CO;
    const int tid = threadIdx.x;
    const int r0 = tid / CO;
    const int c = 2 * (tid - r0 * CO);
    if (r0 >= RPP) return;
    const bool second = c + 1 < ncols;
#pragma unroll 4
    for (int r = r0; r < nrows; r += RPP) {
        T a = tile[r * opitch + c];
        T b = tile[r * opitch + c + 1];
        if constexpr (ACC) {   // accumulate into what an earlier launch stored
            a += dst[(int64_t)r * N + c];
            if (second) b += dst[(int64_t)r * N + c + 1];
        }
        store_out(dst + (int64_t)r * N + c, a);
        if (second) store_out(dst + (int64_t)r * N + c + 1, b);
    }
}

// Stage epilogue, split in two so that a lane issues the loads of a batch of
// nodes before any of their stores (the state pointers may alias as far as
// the compiler knows, so a store would otherwise hold back every later load).
// rk_load: u0 and acc_in of state field t at node offset node (relative to the
// pass's interior origin).  rk_store: stage = u0 + a k, acc = acc_in + b k,
// and with a lattice the face ghosts of the next state; (x, y, z) are the
// node's coordinates in the block.  Same arithmetic as the separate stage
// kernel.
template <typename T>
__device__ __forceinline__ void rk_load(const RkArgs &rk, const PassDesc &pd, int t, int64_t node, T &v, T &ai) {
    const int64_t idx = pd.in_base + (int64_t)t * pd.in_fstride + node;
    v = T(0);
    if (rk.stage || rk.acc_is_u0) v = static_cast<const T *>(rk.u0)[idx];
    ai = rk.acc_is_u0 ? v : static_cast<const T *>(rk.acc_in)[idx];
}

// Ghost targets of one block for the stage epilogue: per face (x-, x+, y-,
// y+, z-, z+) the offset that takes a node's offset within this block's
// storage to the facing ghost node in the neighbour's storage.  Read once per
// item (the block is the item's).
struct RkGhost {
    int64_t base[6];
    bool on;
};

__device__ __forceinline__ RkGhost rk_ghost(const RkArgs &rk, const EpiDesc &ed) {
    RkGhost g;
    g.on = rk.lat[0] > 0;
    if (!g.on) return g;
    const int bx = rk.lat[0], by = rk.lat[1], bz = rk.lat[2];
    const int kx = ed.block % bx, ky = (ed.block / bx) % by, kz = ed.block / (bx * by);
    const int64_t sy = (int64_t)ed.n[1] * ed.sy, sz = (int64_t)ed.n[2] * ed.sz;
    g.base[0] = rk.in_off[(kz * by + ky) * bx + (kx + bx - 1) % bx] + ed.n[0];
    g.base[1] = rk.in_off[(kz * by + ky) * bx + (kx + 1) % bx] - ed.n[0];
    g.base[2] = rk.in_off[(kz * by + (ky + by - 1) % by) * bx + kx] + sy;
    g.base[3] = rk.in_off[(kz * by + (ky + 1) % by) * bx + kx] - sy;
    g.base[4] = rk.in_off[(((kz + bz - 1) % bz) * by + ky) * bx + kx] + sz;
    g.base[5] = rk.in_off[(((kz + 1) % bz) * by + ky) * bx + kx] - sz;
    return g;
}

template <typename T>
__device__ __forceinline__ void rk_store(const RkArgs &rk, const EpiDesc &ed, const RkGhost &gh, const PassDesc &pd,
                                         int t, int64_t node, int x, int y, int z, T v, T ai, T k) {
    const int64_t idx = pd.in_base + (int64_t)t * pd.in_fstride + node;
    const T sv = v + (T)rk.a * k, av = ai + (T)rk.b * k;
    if (rk.stage) static_cast<T *>(rk.stage)[idx] = sv;
    static_cast<T *>(rk.acc)[idx] = av;
    if (gh.on) {
        const T nv = rk.stage ? sv : av;
        T *next = static_cast<T *>(rk.stage ? rk.stage : rk.acc);
        const int64_t here = ed.org + (int64_t)t * pd.in_fstride + node;   // within the block's storage
        const int ng = ed.ng;
        if (x < ng) next[gh.base[0] + here] = nv;
        if (x >= ed.n[0] - ng) next[gh.base[1] + here] = nv;
        if (y < ng) next[gh.base[2] + here] = nv;
        if (y >= ed.n[1] - ng) next[gh.base[3] + here] = nv;
        if (z < ng) next[gh.base[4] + here] = nv;
        if (z >= ed.n[2] - ng) next[gh.base[5] + here] = nv;
    }
}

// k of a stage epilogue: the addends stored at output offset oo (within the
// block), in order, then the derivative.
template <typename T>
__device__ __forceinline__ T rk_k(const EpiDesc &ed, const T *out, int64_t oo, T d) {
    if (ed.nadd == 0) return d;
    T s = out[ed.add[0] + oo];
    if (ed.nadd > 1) s = s + out[ed.add[1] + oo];
    return s + d;
}

// Nodes per load batch of the stage epilogue (more batches in flight cost
// registers, and with them waves per SIMD).
constexpr int kRkBatch = 4;

// x lines of a stage epilogue: the results staged in the tile (row r = line
// line0 + r, columns col0 .. col0 + ncols - 1 of the line, pitch opitch) go
// into the stage update instead of the output.  Thread tid owns node pair
// tid % CO of rows tid / CO + k * RPP, as in store_x, kRkBatch / 2 rows per
// load batch.
template <typename T, int WG>
__device__ __forceinline__ void store_x_rk(const RkArgs &rk, const EpiDesc &ed, const PassDesc &pd, const T *out,
                                           const T *tile, int line0, int nrows, int col0, int ncols, int opitch) {
    constexpr int NT = 64 * WG;
    constexpr int RB = kRkBatch / 2;
    const int CO = (ncols + 1) >> 1;
    const int RPP = NT / CO;
    const int tid = threadIdx.x;
    const int r0 = tid / CO;
    const int c = 2 * (tid - r0 * CO);
    if (r0 >= RPP) return;
    const bool second = c + 1 < ncols;
    const RkGhost gh = rk_ghost(rk, ed);
    for (int rb = r0; rb < nrows; rb += RB * RPP) {
        T v[RB][2], ai[RB][2], k[RB][2];
        int64_t node[RB];
        int lu[RB], lv[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = rb + q * RPP;
            if (r >= nrows) continue;
            const int line = line0 + r;
            lu[q] = line % pd.nu;
            lv[q] = line / pd.nu;
            node[q] = (int64_t)lv[q] * pd.sv + (int64_t)lu[q] * pd.su + col0 + c;
            const int64_t oo = (int64_t)line * pd.N + col0 + c;
            rk_load<T>(rk, pd, ed.tgt, node[q], v[q][0], ai[q][0]);
            k[q][0] = rk_k<T>(ed, out, oo, tile[r * opitch + c]);
            if (second) {
                rk_load<T>(rk, pd, ed.tgt, node[q] + 1, v[q][1], ai[q][1]);
                k[q][1] = rk_k<T>(ed, out, oo + 1, tile[r * opitch + c + 1]);
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (rb + q * RPP >= nrows) continue;
            rk_store<T>(rk, ed, gh, pd, ed.tgt, node[q], col0 + c, lu[q], lv[q], v[q][0], ai[q][0], k[q][0]);
            if (second)
                rk_store<T>(rk, ed, gh, pd, ed.tgt, node[q] + 1, col0 + c + 1, lu[q], lv[q], v[q][1], ai[q][1],
                            k[q][1]);
        }
    }
}

// Item body for one compiled partition length L.
template <typename T, int NL, int NOPS, int PAR, int MI, int HW, int L, bool PAD, bool CHK, int XM, int WG>
__device__ __forceinline__ void run_item(LineCtx<T> &c, const WorkItem &wi, T *out, bool xdir, bool active,
                                         int lu, int lv, const RkArgs &rk) {
    const PassDesc &pd = *c.pd;
    // stage epilogue (mode 2 classes, single operator): the pass folds its
    // derivative into a state update instead of storing it
    bool epi = false;
    const EpiDesc *ed = nullptr;
    if constexpr (XM == 2) {
        ed = rk.epi + wi.pass;
        epi = ed->mode == 1;
    }
    T y[NOPS][L];
    if (xdir) {
        // the tile holds one column chunk (P/C partitions and the halo) at a
        // time: stage it, the waves of that chunk read their inputs, next chunk
        const int nsub = WG / c.P;
        const int nrows_all = nsub * 64;
        const int N = pd.N;
        const int C = CHK ? c.C : 1;
        const int PC = c.P / C;
        T fin[L + 2 * HW];
        if constexpr (CHK) {   // classes with long partitions: any number of chunks
            for (int ch = 0; ch < C; ++ch) {
                if (ch > 0) __syncthreads();   // the previous chunk's readers are done
                stage_x<T, HW, WG>(pd, c.fbase, c.line0, nrows_all, ch * PC * L - HW, PC * L + 2 * HW, c.tile,
                                   c.tpitch, c.periodic);
                __syncthreads();
                if (c.chunk == ch) {
                    const int k0 = (c.p - ch * PC) * L;
#pragma unroll
                    for (int t = 0; t < L + 2 * HW; ++t) fin[t] = c.tile[c.trow * c.tpitch + k0 + t];
                }
            }
        } else {   // one chunk: the whole line, staged by the kernel before dispatch
#pragma unroll
            for (int t = 0; t < L + 2 * HW; ++t) fin[t] = c.tile[c.trow * c.tpitch + c.p * L + t];
        }
        solve_partition<T, NL, NOPS, PAR, MI, HW, L, true, PAD, XM>(c, y, fin);
        // results back through the tile, chunk by chunk, then contiguous
        // coalesced stores: x-lines line0.. of one field are consecutive rows
        // of the interior output
        if constexpr (CHK) {
            const int opitch = (PC * L) | 1;
            int nrows = pd.nlines - wi.line0;
            if (nrows > nrows_all) nrows = nrows_all;
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                T *dst = out + pd.out_base[o] + (int64_t)wi.field * pd.out_fstride + (int64_t)wi.line0 * N;
                for (int ch = 0; ch < C; ++ch) {
                    __syncthreads();   // every lane is done with the input / previous chunk in the tile
                    if (c.chunk == ch) {
                        const int k0 = (c.p - ch * PC) * L;
#pragma unroll
                        for (int i = 0; i < L; ++i)
                            if (c.p * L + i < N) c.tile[c.trow * opitch + k0 + i] = y[o][i];
                    }
                    __syncthreads();
                    const int col0 = ch * PC * L;
                    const int ncols = min(N - col0, PC * L);
                    if (ncols > 0) {
                        if (epi)
                            store_x_rk<T, WG>(rk, *ed, pd, out, c.tile, wi.line0, nrows, col0, ncols, opitch);
                        else
                            store_x<T, WG, XM == 3>(dst + col0, c.tile, nrows, N, ncols, opitch);
                    }
                }
            }
        } else {
            const int opitch = N | 1;
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                __syncthreads();   // every lane is done with the input / previous op in the tile
#pragma unroll
                for (int i = 0; i < L; ++i)
                    if (c.p * L + i < N) c.tile[c.trow * opitch + c.p * L + i] = y[o][i];
                __syncthreads();
                T *dst = out + pd.out_base[o] + (int64_t)wi.field * pd.out_fstride + (int64_t)wi.line0 * N;
                int nrows = pd.nlines - wi.line0;
                if (nrows > nrows_all) nrows = nrows_all;
                if (epi)
                    store_x_rk<T, WG>(rk, *ed, pd, out, c.tile, wi.line0, nrows, 0, N, opitch);
                else
                    store_x<T, WG, XM == 3>(dst, c.tile, nrows, N, N, opitch);
            }
        }
    } else {
        T fin[L + 2 * HW];
        solve_partition<T, NL, NOPS, PAR, MI, HW, L, false, PAD, XM>(c, y, fin);
        if constexpr (XM == 2) {
            if (epi && active) {
                // node (lu, lv, j) of the line in the block: coordinates by direction
                const int nreal = pd.N - c.p * L;
                const int64_t node0 = (int64_t)lv * pd.sv + (int64_t)lu * pd.su + (int64_t)c.p * L * pd.sd;
                const int64_t oo0 = (int64_t)lv * pd.osv + (int64_t)lu * pd.osu + (int64_t)c.p * L * pd.osd;
                const bool self = ed->self_tgt >= 0;
                const RkGhost gh = rk_ghost(rk, *ed);
                // x and (y or z) of the lane's nodes: lu is x for y and z lines;
                // the other coordinate is lv, the line's own is j
                const int dir = ed->dir;
                // the operator's field (k = derivative and addends), then the
                // line's own field (k = its value) if the pass updates one
#pragma unroll
                for (int pass2 = 0; pass2 < 2; ++pass2) {
                    if (pass2 == 1 && !self) break;
                    const int t = pass2 ? ed->self_tgt : ed->tgt;
#pragma unroll
                    for (int i0 = 0; i0 < L; i0 += kRkBatch) {
                        constexpr int RB = kRkBatch;
                        T v[RB], ai[RB], k[RB];
#pragma unroll
                        for (int q = 0; q < RB; ++q) {
                            const int i = i0 + q;
                            if (i >= L || (PAD && i >= nreal)) continue;
                            rk_load<T>(rk, pd, t, node0 + (int64_t)i * pd.sd, v[q], ai[q]);
                            k[q] = pass2 ? fin[HW + i] : rk_k<T>(*ed, out, oo0 + (int64_t)i * pd.osd, y[0][i]);
                        }
#pragma unroll
                        for (int q = 0; q < RB; ++q) {
                            const int i = i0 + q;
                            if (i >= L || (PAD && i >= nreal)) continue;
                            const int j = c.p * L + i;
                            rk_store<T>(rk, *ed, gh, pd, t, node0 + (int64_t)i * pd.sd, lu, dir == 1 ? j : lv,
                                        dir == 2 ? j : lv, v[q], ai[q], k[q]);
                        }
                    }
                }
            }
        }
        if (active && !epi) {
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                T *dst = out + pd.out_base[o] + (int64_t)wi.field * pd.out_fstride + (int64_t)lv * pd.osv +
                         (int64_t)lu * pd.osu + (int64_t)c.p * L * pd.osd;
                const int64_t osd = pd.osd;
                const int nreal = pd.N - c.p * L;   // rows of this partition inside the line
                if constexpr (XM == 3) {
                    // accumulate, in batches: a batch's earlier values are all loaded
                    // before its stores (which may alias them as far as the compiler
                    // knows), without holding a whole partition of them at once
                    constexpr int RB = 4;
#pragma unroll
                    for (int i0 = 0; i0 < L; i0 += RB) {
                        T prev[RB];
#pragma unroll
                        for (int q = 0; q < RB; ++q)
                            if (i0 + q < L && (!PAD || i0 + q < nreal)) prev[q] = dst[(int64_t)(i0 + q) * osd];
#pragma unroll
                        for (int q = 0; q < RB; ++q)
                            if (i0 + q < L && (!PAD || i0 + q < nreal))
                                store_out(dst + (int64_t)(i0 + q) * osd, y[o][i0 + q] + prev[q]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < L; ++i) {
                        if (!PAD || i < nreal) store_out(dst, y[o][i]);
                        dst += osd;
                    }
                }
            }
        }
    }
    __syncthreads();   // LDS (tile and exchange) is reused by the next item
}

template <int... Ls>
struct LSet {
    static constexpr int n = sizeof...(Ls);
};

template <typename T, int NL, int NOPS, int PAR, int MI, int HW, bool CHK, int XM, int WG, int L0, int... Ls>
__device__ __forceinline__ void dispatch_L(int lcode, bool pad, LineCtx<T> &c, const WorkItem &wi, T *out,
                                           bool xdir, bool active, int lu, int lv, const RkArgs &rk) {
    if (lcode == 0) {
        if (pad)
            run_item<T, NL, NOPS, PAR, MI, HW, L0, true, CHK, XM, WG>(c, wi, out, xdir, active, lu, lv, rk);
        else
            run_item<T, NL, NOPS, PAR, MI, HW, L0, false, CHK, XM, WG>(c, wi, out, xdir, active, lu, lv, rk);
        return;
    }
    if constexpr (sizeof...(Ls) > 0)
        dispatch_L<T, NL, NOPS, PAR, MI, HW, CHK, XM, WG, Ls...>(lcode - 1, pad, c, wi, out, xdir, active, lu, lv,
                                                                 rk);
}

// Classes whose partitions reach this many rows stage long x lines in column
// chunks (the host sets C > 1 only for them).
constexpr int kChunkMinL = 48;

template <int... Ls>
constexpr int max_L() {
    int m = 0;
    for (int v : {Ls...}) m = v > m ? v : m;
    return m;
}

// Persistent line kernel: every workgroup walks the work list with a grid
// stride.  Work item meta: P in bits 0..3, index of L in the compiled set in
// bits 4..7, x lines: column chunks - 1 in bits 8..9.  Dynamic LDS: exchange
// area and x tile (one column chunk), overlaid.  XM (extension mode): 1
// iterated closures, with each line's two end values per op read from ev; 2
// stage epilogue of the passes whose EpiDesc asks for it (rk); 3 accumulate:
// the derivative is added to what the output already holds (the second
// order of a symmetrised mixed derivative, after a launch stored the first).
template <typename T, int NL, int NOPS, int PAR, int MI, int HW, int XM, int WG, int... Ls>
__global__ void __launch_bounds__(64 * WG)
k_lines(const WorkItem *__restrict__ items, int nitems, const int *__restrict__ qoff,
        const PassDesc *__restrict__ passes, const T *__restrict__ tabs, const int64_t *__restrict__ taboff,
        const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ ev, const RkArgs rk) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *exch = reinterpret_cast<T *>(smem_raw);
    constexpr int kLs[] = {Ls...};
    constexpr bool kChunked = max_L<Ls...>() >= kChunkMinL;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = threadIdx.x & 63;

    // Work distribution.  Plain: grid-stride over the list (with one workgroup
    // per item, the host may have ordered the list so that item b belongs to
    // XCD b % kXCD; padding items have pass -1).  XCD-aware persistent grid
    // (qoff given, grid a multiple of kXCD): workgroup ids are dealt
    // round-robin to the XCDs, so workgroup b runs on XCD b % kXCD and takes
    // the items of queue b % kXCD; each queue holds whole block-fields, whose
    // x/y/z passes then share one XCD's L2.
    int it = blockIdx.x, it_end = nitems, stride = gridDim.x;
    if (qoff && qoff[0] < 0) {
        // one workgroup per item, list in XCD-interleaved order (position 8 r + k
        // holds queue k's r-th item; length a multiple of 8).  A launch's
        // workgroups are dealt round-robin to the XCDs from a launch-dependent
        // start, so workgroup b takes the item of its group of 8 that belongs to
        // the XCD it runs on (read from the hardware): a permutation within the
        // group, and the same XCD for a block-field in every launch.
        const int xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kXCD - 1);   // HW_REG_XCC_ID
        it = (int)(blockIdx.x & ~(unsigned)(kXCD - 1)) + xcc;
        it_end = it + 1;
        stride = 1;
    } else if (qoff) {
        const int q = blockIdx.x % kXCD;
        it = qoff[q] + blockIdx.x / kXCD;
        it_end = qoff[q + 1];
        stride = gridDim.x / kXCD;
    }
    for (; it < it_end; it += stride) {
        const WorkItem wi = items[it];
        if (wi.pass < 0) continue;   // padding of the XCD-interleaved order
        const PassDesc &pd = passes[wi.pass];
        LineCtx<T> c;
        c.pd = &pd;
        c.P = wi.meta & 15;
        const int lcode = (wi.meta >> 4) & 15;
        c.sub = w / c.P;
        c.p = w - c.sub * c.P;
        c.g = g;
        c.periodic = pd.periodic != 0;
        c.exch = exch;
#pragma unroll
        for (int o = 0; o < NOPS; ++o) c.tb[o] = tabs + taboff[pd.tab[o]];
        const bool xdir = pd.sd == 1;
        int line = wi.line0 + c.sub * 64 + g;
        const bool active = line < pd.nlines;
        if (!active) line = pd.nlines - 1;
        if constexpr (XM == 1) {
#pragma unroll
            for (int o = 0; o < NOPS; ++o) {
                const T *e = ev + pd.ev_base[o] + ((int64_t)wi.field * pd.nlines + line) * 2;
                c.em[o] = e[0];
                c.ep[o] = e[1];
            }
        }
        const int lu = line % pd.nu;
        const int lv = line / pd.nu;
        const T *fbase = in + pd.in_base + (int64_t)(pd.field0 + wi.field) * pd.in_fstride;
        if (xdir) {
            T *tile = exch;   // shared with the exchange area
            c.tile = tile;
            c.trow = c.sub * 64 + g;
            if constexpr (kChunked) {   // staged chunk by chunk in the item body
                c.C = ((wi.meta >> 8) & 3) + 1;
                const int PC = c.P / c.C;
                c.chunk = c.p / PC;
                c.tpitch = (PC * kLs[lcode] + 2 * HW) | 1;
                c.fbase = fbase;
                c.line0 = wi.line0;
            } else {
                const int Npad = c.P * kLs[lcode];
                c.C = 1;
                c.chunk = 0;
                c.tpitch = (Npad + 2 * HW) | 1;
                stage_x<T, HW, WG>(pd, fbase, wi.line0, (WG / c.P) * 64, -HW, Npad + 2 * HW, tile, c.tpitch,
                                   c.periodic);
                __syncthreads();
            }
        } else {
            c.src = fbase + (int64_t)lv * pd.sv + (int64_t)lu * pd.su;
        }
        const bool pad = c.P * kLs[lcode] != pd.N;
        dispatch_L<T, NL, NOPS, PAR, MI, HW, kChunked, XM, WG, Ls...>(lcode, pad, c, wi, out, xdir, active, lu, lv, rk);
    }
}

}  // namespace cfd
