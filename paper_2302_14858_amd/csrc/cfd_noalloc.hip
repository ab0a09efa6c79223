// Allocation-free apply: one operator along one direction on every line of
// one block, with nothing allocated on the device.
//
// cfd_plan_create allocates a plan's device tables and, while it builds them,
// a scratch area for the FP64 factorisation kernel.  Callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses that
// forbid it) use cfd_apply_block_noalloc instead: the solve tables, the pass
// descriptor, the work list and the factorisation scratch all live in the
// file-scope device array `scratch` below, and every step (filling those
// records, building the tables in FP64, the FP32 copy, the line kernel) is a
// kernel launch on the caller's stream.  The line kernel and the table builder
// are the ones plans use, with the same partition choice, so the result equals
// that of a plan with the same single operator bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "cfd_internal.h"
#include "cfd_kernels_reg.h"

namespace cfd {
constexpr size_t kNoAllocBytes = size_t(8) << 20;   // size of the scratch array
constexpr int kNoAllocMaxDevices = 64;
}  // namespace cfd

// Device scratch of the allocation-free apply: tables, records and work list
// of the current call.  Each GPU holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[cfd::kNoAllocBytes];

namespace cfd {
namespace {

// Records the set-up kernel writes, passed by value.
struct SetupArgs {
    double coef[kCoefHdr];     // coefficient block of the table
    unsigned char spec[128];   // table-builder spec (TabSpec bytes)
    PassDesc pd;
    int32_t meta;              // work-item meta (P, L index, x chunks)
    int32_t nitems, items_per_field, lines_per_item;
    double *tab;               // destinations inside the scratch array
    unsigned char *spec_dst;
    PassDesc *pd_dst;
    int64_t *taboff;
    int *status;
    WorkItem *items;
};

__global__ void k_noalloc_setup(SetupArgs a) {
    const int t = threadIdx.x + blockIdx.x * blockDim.x;
    const int nt = blockDim.x * gridDim.x;
    for (int i = t; i < kCoefHdr; i += nt) a.tab[i] = a.coef[i];
    for (int i = t; i < (int)sizeof(a.spec); i += nt) a.spec_dst[i] = a.spec[i];
    if (t == 0) {
        *a.pd_dst = a.pd;
        a.taboff[0] = 0;
        a.status[0] = 0;
    }
    for (int i = t; i < a.nitems; i += nt) {
        WorkItem w;
        w.pass = 0;
        w.field = i / a.items_per_field;
        w.line0 = (i - w.field * a.items_per_field) * a.lines_per_item;
        w.meta = a.meta;
        a.items[i] = w;
    }
}

cfd_status nfail(cfd_status st, const std::string &m) { return set_error(st, m); }

// Address of this device's copy of `scratch`, looked up once per device with
// that device current.  The array's name is a host-side stand-in: only this
// address may be passed to kernels.
void *scratch_ptr(int dev, hipError_t &err) {
    static std::mutex mu;
    static void *ptr[kNoAllocMaxDevices] = {};
    err = hipSuccess;
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace
}  // namespace cfd

using namespace cfd;

extern "C" cfd_status cfd_apply_block_noalloc(const cfd_scheme *sc, const cfd_block *blk, int dir, int nfields,
                                              int field, cfd_dtype dtype, const void *in_dev, void *out_dev,
                                              void *stream) {
    if (!sc || !blk || !in_dev || !out_dev) return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: null argument");
    if (dir < 0 || dir > 2) return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: direction not in 0..2");
    if (sc->s.kind != 0)
        return nfail(CFD_EUNSUPPORTED, "cfd_apply_block_noalloc: biased schemes need a plan (cfd_plan_create)");
    if (nfields < 1 || field < -1 || field >= nfields)
        return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: bad field count or field index");
    if (dtype != CFD_F64 && dtype != CFD_F32)
        return nfail(dtype == CFD_MIXED_BF16 ? CFD_EUNSUPPORTED : CFD_EINVAL,
                     "cfd_apply_block_noalloc: dtype must be CFD_F64 or CFD_F32");
    if (((uintptr_t)in_dev % 16) || ((uintptr_t)out_dev % 16))
        return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: buffers must be 16-byte aligned");
    const cfd_block &b = *blk;
    for (int d = 0; d < 3; ++d) {
        if (b.n[d] < 1) return nfail(CFD_ESHAPE, "cfd_apply_block_noalloc: block extent < 1");
        if (!(b.h[d] > 0)) return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: grid spacing must be positive");
        if (b.boundary[d] != CFD_BOUNDARY_CLOSURE && b.boundary[d] != CFD_BOUNDARY_PERIODIC)
            return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: unknown boundary kind");
    }
    if (b.ng < 0) return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: negative ghost width");
    const Scheme &s = sc->s;
    const int per = b.boundary[dir] == CFD_BOUNDARY_PERIODIC;
    const int N = b.n[dir];
    if (b.ng < required_ghosts(s, per)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "cfd_apply_block_noalloc: scheme '%s' needs %d ghost layers, block has %d",
                      s.name.c_str(), required_ghosts(s, per), b.ng);
        return nfail(CFD_EGHOST, buf);
    }
    if (!per && s.nl > 0 && N < 2 * s.nc + 1)
        return nfail(CFD_ESHAPE, "cfd_apply_block_noalloc: line too short for the closure rows");
    if (per && N < std::max(2 * s.nl + 1, std::max(s.m, s.mc)))
        return nfail(CFD_ESHAPE, "cfd_apply_block_noalloc: periodic line shorter than the stencil");
    const int64_t ng = b.ng;
    const int64_t fin = (b.n[0] + 2 * ng) * (b.n[1] + 2 * ng) * (b.n[2] + 2 * ng);
    if (fin * nfields > (int64_t(1) << 40)) return nfail(CFD_EINVAL, "cfd_apply_block_noalloc: layout too large");

    const bool f32 = dtype == CFD_F32;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    int max_lds = 65536;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nfail(CFD_EDEVICE, std::string("cfd_apply_block_noalloc: ") + hipGetErrorString(e));
    }

    // the pass and its schedule: the default partition choice of a plan
    PassHost ps;
    ps.block = 0;
    ps.dir = dir;
    ps.field0 = field < 0 ? 0 : field;
    ps.nfield = field < 0 ? nfields : 1;
    ps.nops = 1;
    ps.N = N;
    ps.ng = b.ng;
    ps.periodic = per;
    ps.nl = s.nl;
    ps.par = (s.d % 2) ? 1 : 0;
    ps.mi = s.m;
    ps.hw = std::max(s.m, per ? 0 : s.mc);
    int cands[4];
    if (candidate_Ps(ps, f32, (size_t)max_lds, cands) == 0)
        return nfail(CFD_EUNSUPPORTED, "cfd_apply_block_noalloc: no compiled line kernel for this line length");
    place_pass(ps, f32, cands[0]);
    const size_t lds = pass_lds(ps, f32);

    // scratch layout: FP64 table, FP32 table, factorisation scratch, records, work list
    const int Npad = ps.P * ps.L;
    const int64_t tel = (table_elems(Npad, ps.P, s.nl) + 7) & ~int64_t(7);
    const int64_t bscr = tab_scratch(ps.P, ps.L, s.nl);
    const int per_item = kWave * (waves_for(ps.P) / ps.P);
    const int64_t nlines = (int64_t)b.n[dir == 0 ? 1 : 0] * b.n[dir == 2 ? 1 : 2];
    const int64_t items_per_field = (nlines + per_item - 1) / per_item;
    const int64_t nitems = items_per_field * ps.nfield;
    size_t off = 0;
    const size_t o_tab64 = off;
    off = align256(off + tel * sizeof(double));
    const size_t o_tab32 = off;
    if (f32) off = align256(off + tel * sizeof(float));
    const size_t o_bscr = off;
    off = align256(off + bscr * sizeof(double));
    const size_t o_spec = off;
    off = align256(off + 128);
    const size_t o_pd = off;
    off = align256(off + sizeof(PassDesc));
    const size_t o_taboff = off;
    off = align256(off + sizeof(int64_t));
    const size_t o_status = off;
    off = align256(off + sizeof(int));
    const size_t o_items = off;
    if (nitems > INT32_MAX / 2) return nfail(CFD_EUNSUPPORTED, "cfd_apply_block_noalloc: too many lines");
    off = align256(off + (size_t)nitems * sizeof(WorkItem));
    if (off > kNoAllocBytes) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "cfd_apply_block_noalloc: needs %zu bytes of device scratch, the limit is %zu "
                      "(fewer fields or lines per call)", off, kNoAllocBytes);
        return nfail(CFD_EUNSUPPORTED, buf);
    }
    if (tabspec_size() > sizeof(SetupArgs::spec))
        return nfail(CFD_EDEVICE, "cfd_apply_block_noalloc: table spec record does not fit");

    unsigned char *base = (unsigned char *)scratch_ptr(dev, e);
    if (!base) {
        (void)hipGetLastError();
        return nfail(CFD_EDEVICE, std::string("cfd_apply_block_noalloc: scratch address: ") + hipGetErrorString(e));
    }

    SetupArgs a;
    std::memset(&a, 0, sizeof a);
    fill_coef_block(a.coef, s);
    fill_tabspec(a.spec, N, ps.P, ps.L, s.nl, per ? 0 : s.nc, per, s.lhs, 0, s.ext, s.cl_d0, s.cl_up,
                 s.gamma);   // real length; rows >= N are padding
    {
        const int64_t ob[2] = {0, 0};
        const int tab[2] = {0, 0};
        const double hinv[2] = {1.0 / std::pow(b.h[dir], scale_power(s)), 0.0};
        fill_pass_desc(a.pd, b, 0, ps, ob, tab, hinv);
    }
    a.meta = ps.P | (ps.lcode << 4) | ((ps.C - 1) << 8);
    a.nitems = (int32_t)nitems;
    a.items_per_field = (int32_t)items_per_field;
    a.lines_per_item = per_item;
    a.tab = (double *)(base + o_tab64);
    a.spec_dst = base + o_spec;
    a.pd_dst = (PassDesc *)(base + o_pd);
    a.taboff = (int64_t *)(base + o_taboff);
    a.status = (int *)(base + o_status);
    a.items = (WorkItem *)(base + o_items);

    hipStream_t st = (hipStream_t)stream;
    const int sgrid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nitems + 255) / 256));
    hipLaunchKernelGGL(k_noalloc_setup, dim3(sgrid), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = launch_build_tables(1, a.spec_dst, a.tab, (double *)(base + o_bscr), bscr, a.status, st);
    void *tabs = a.tab;
    if (e == hipSuccess && f32) {
        e = launch_to_f32(tel, a.tab, (float *)(base + o_tab32), st);
        tabs = base + o_tab32;
    }
    if (e == hipSuccess && nitems > 0)
        e = launch_lines(ps.cls->fn, ps.cls->wg, (int)nitems, lds, st, a.items, (int)nitems, nullptr, a.pd_dst, tabs, a.taboff,
                         in_dev, out_dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nfail(CFD_EDEVICE, std::string("cfd_apply_block_noalloc: launch: ") + hipGetErrorString(e));
    }
    return CFD_OK;
}

