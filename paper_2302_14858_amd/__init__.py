"""Python binding of the MI355X compact finite-difference library.

Thin wrappers over the C ABI (include/cfd.h) with the same names; device
memory and streams come from torch (ROCm).  Every derivative is computed by
the HIP kernels in libcfd_mi355x.so; there is no CPU path, and the binding
raises if the library is missing.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

from . import _lib
from ._lib import (CFD_BOUNDARY_CLOSURE, CFD_BOUNDARY_PERIODIC, CFD_F32, CFD_F64, CFD_MIXED_BF16, CfdError,
                   check, lib)

__all__ = ["Scheme", "Plan", "cfd_abi_version", "cfd_taylor_scheme", "cfd_axpby", "cfd_xpcy", "CfdError", "CFD_F64", "CFD_F32",
           "CFD_MIXED_BF16", "CFD_BOUNDARY_CLOSURE", "CFD_BOUNDARY_PERIODIC"]


def cfd_abi_version() -> int:
    return lib().cfd_abi_version()


def cfd_taylor_scheme(dr: int, L: int, R: int, classes: Sequence) -> Dict:
    """Fully determined multi-derivative scheme: classes is a list of (d_I, L_k, R_k)."""
    n = len(classes)
    dI = (ctypes.c_int * n)(*[c[0] for c in classes])
    Lk = (ctypes.c_int * n)(*[c[1] for c in classes])
    Rk = (ctypes.c_int * n)(*[c[2] for c in classes])
    cap = (L + R + 1) + sum(c[1] + c[2] + 1 for c in classes)
    coef = (ctypes.c_double * cap)()
    order = ctypes.c_int()
    check(lib().cfd_taylor_scheme(dr, L, R, n, dI, Lk, Rk, coef, cap, ctypes.byref(order)))
    vals = list(coef)
    out = {"order": order.value, "lhs": vals[:L + R + 1], "rhs": []}
    pos = L + R + 1
    for c in classes:
        w = c[1] + c[2] + 1
        out["rhs"].append(vals[pos:pos + w])
        pos += w
    return out


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Scheme:
    """A compact finite-difference scheme (library-owned handle)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def cfd_scheme_named(cls, name: str) -> "Scheme":
        out = ctypes.c_void_p()
        check(lib().cfd_scheme_named(name.encode(), ctypes.byref(out)))
        return cls(out.value)

    named = cfd_scheme_named

    @classmethod
    def cfd_scheme_design(cls, d: int, order: int, nl: int, m: int, eta_c: float = 1.0, closure_mc: int = 0,
                          matched: bool = True) -> "Scheme":
        out = ctypes.c_void_p()
        check(lib().cfd_scheme_design(d, order, nl, m, float(eta_c), closure_mc, int(matched), ctypes.byref(out)))
        return cls(out.value)

    design = cfd_scheme_design

    @classmethod
    def cfd_scheme_create(cls, d: int, order: int, lhs: Sequence[float], rhs: Sequence[float],
                          closure: Sequence[Sequence[float]] = ()) -> "Scheme":
        nl = (len(lhs) - 1) // 2
        m = (len(rhs) - 1) // 2
        nc = len(closure)
        mc = (len(closure[0]) - 1) // 2 if nc else 0
        L = (ctypes.c_double * len(lhs))(*lhs)
        R = (ctypes.c_double * len(rhs))(*rhs)
        flat = [v for row in closure for v in row] or [0.0]
        C = (ctypes.c_double * len(flat))(*flat)
        out = ctypes.c_void_p()
        check(lib().cfd_scheme_create(d, order, nl, L, m, R, nc, mc, C, ctypes.byref(out)))
        return cls(out.value)

    create = cfd_scheme_create

    def cfd_scheme_get(self) -> Dict:
        ints = [ctypes.c_int() for _ in range(6)]
        lhs = (ctypes.c_double * 5)()
        rhs = (ctypes.c_double * 11)()
        cl = (ctypes.c_double * 22)()
        check(lib().cfd_scheme_get(self._h, *[ctypes.byref(v) for v in ints], lhs, rhs, cl))
        d, order, nl, m, nc, mc = (v.value for v in ints)
        return {"d": d, "order": order, "nl": nl, "m": m, "nc": nc, "mc": mc, "lhs": list(lhs), "rhs": list(rhs),
                "closure": [list(cl[0:11]), list(cl[11:22])]}

    get = cfd_scheme_get

    @classmethod
    def cfd_scheme_design_biased(cls, family: str, M: int, lam: float = 0.0, bias: int = -1) -> "Scheme":
        out = ctypes.c_void_p()
        check(lib().cfd_scheme_design_biased(family.encode(), M, float(lam), int(bias), ctypes.byref(out)))
        return cls(out.value)

    design_biased = cfd_scheme_design_biased

    @classmethod
    def cfd_scheme_dissipation(cls, r: int, sigma: float) -> "Scheme":
        out = ctypes.c_void_p()
        check(lib().cfd_scheme_dissipation(int(r), float(sigma), ctypes.byref(out)))
        return cls(out.value)

    dissipation = cfd_scheme_dissipation

    def cfd_scheme_get_biased(self) -> Dict:
        bias, order, alpha = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        a = (ctypes.c_double * 11)()
        c = (ctypes.c_double * 12)()
        check(lib().cfd_scheme_get_biased(self._h, ctypes.byref(bias), ctypes.byref(order), ctypes.byref(alpha),
                                          a, c))
        return {"bias": bias.value, "order": order.value, "alpha": alpha.value, "a": list(a), "c": list(c)}

    get_biased = cfd_scheme_get_biased

    def cfd_scheme_get_embedded(self) -> Dict:
        a2, m2 = ctypes.c_double(), ctypes.c_int()
        check(lib().cfd_scheme_get_embedded(self._h, ctypes.byref(a2), ctypes.byref(m2)))
        return {"alpha2": a2.value, "M": m2.value}

    get_embedded = cfd_scheme_get_embedded

    def cfd_scheme_required_ghosts(self, boundary: int = CFD_BOUNDARY_CLOSURE) -> int:
        ng = ctypes.c_int()
        check(lib().cfd_scheme_required_ghosts(self._h, boundary, ctypes.byref(ng)))
        return ng.value

    required_ghosts = cfd_scheme_required_ghosts

    def __del__(self):
        try:
            if self._h:
                lib().cfd_scheme_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


class Plan:
    """A batch of blocks x fields x operators applied in one step.

    blocks: list of dicts with keys n (3 ints), ng, h (3 floats), boundary (3 ints),
            optional in_offset / out_offset (elements; default packed).
    ops:    list of (Scheme, dir), (Scheme, dir, field), (Scheme, dir, field, vel_field),
            (Scheme, dir, field, vel_field, dir2) or (..., dir2, aux_field); vel_field (the velocity
            of an upwind pair), dir2 (second direction of a mixed derivative) and aux_field (the
            sampled f'' a U scheme reads) default to -1.
    """

    def __init__(self, blocks: List[Dict], nfields: int, ops: Sequence, dtype: int = CFD_F64, device: int = 0):
        nb = len(blocks)
        arr = (_lib.cfd_block * nb)()
        for i, b in enumerate(blocks):
            arr[i].n = (ctypes.c_int * 3)(*b["n"])
            arr[i].ng = int(b["ng"])
            arr[i].h = (ctypes.c_double * 3)(*b["h"])
            arr[i].boundary = (ctypes.c_int * 3)(*b["boundary"])
            arr[i].in_offset = int(b.get("in_offset", -1))
            arr[i].out_offset = int(b.get("out_offset", -1))
        self._schemes = [op[0] for op in ops]          # keep handles alive
        oarr = (_lib.cfd_op * len(ops))()
        for i, op in enumerate(ops):
            oarr[i].scheme = op[0]._h
            oarr[i].dir = int(op[1])
            oarr[i].field = int(op[2]) if len(op) > 2 else -1
            oarr[i].vel_field = int(op[3]) if len(op) > 3 else -1
            oarr[i].dir2 = int(op[4]) if len(op) > 4 else -1
            oarr[i].aux_field = int(op[5]) if len(op) > 5 else -1
        desc = _lib.cfd_plan_desc(nb, arr, int(nfields), len(ops), oarr, int(dtype), int(device), 0)
        out = ctypes.c_void_p()
        check(lib().cfd_plan_create(ctypes.byref(desc), ctypes.byref(out)))
        self._h = out
        self.nblocks = nb
        self.dtype = dtype

    def cfd_plan_sizes(self):
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        check(lib().cfd_plan_sizes(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    sizes = cfd_plan_sizes

    def cfd_plan_offsets(self):
        a = (ctypes.c_longlong * self.nblocks)()
        b = (ctypes.c_longlong * self.nblocks)()
        check(lib().cfd_plan_offsets(self._h, a, b))
        return list(a), list(b)

    offsets = cfd_plan_offsets

    def cfd_plan_stats(self):
        a, b = ctypes.c_int(), ctypes.c_longlong()
        check(lib().cfd_plan_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    stats = cfd_plan_stats

    def cfd_apply(self, inp, out, stream=None) -> None:
        check(lib().cfd_apply(self._h, _dev_ptr(inp), _dev_ptr(out), _stream_ptr(stream)))

    apply = cfd_apply

    def cfd_plan_capture_graph(self, inp, out, stream=None) -> None:
        check(lib().cfd_plan_capture_graph(self._h, _dev_ptr(inp), _dev_ptr(out), _stream_ptr(stream)))

    capture_graph = cfd_plan_capture_graph

    def cfd_plan_launch_graph(self, stream=None) -> None:
        check(lib().cfd_plan_launch_graph(self._h, _stream_ptr(stream)))

    launch_graph = cfd_plan_launch_graph

    def cfd_plan_graph_status(self) -> int:
        st = ctypes.c_int()
        check(lib().cfd_plan_graph_status(self._h, ctypes.byref(st)))
        return st.value

    graph_status = cfd_plan_graph_status

    def cfd_plan_count_nonfinite(self, out, stream=None) -> int:
        c = ctypes.c_longlong()
        check(lib().cfd_plan_count_nonfinite(self._h, _dev_ptr(out), _stream_ptr(stream), ctypes.byref(c)))
        return c.value

    count_nonfinite = cfd_plan_count_nonfinite

    def cfd_plan_autotune(self, inp, out, cache_path: Optional[str] = None, stream=None) -> None:
        check(lib().cfd_plan_autotune(self._h, _dev_ptr(inp), _dev_ptr(out), _stream_ptr(stream),
                                      cache_path.encode() if cache_path else None))

    autotune = cfd_plan_autotune

    def cfd_plan_set_schedule(self, N: int = 0, xlines: bool = False, partitions: int = 0,
                              persistent: bool = True, split_x: bool = False, xcd: bool = False,
                              concurrent: bool = False) -> None:
        flags = ((_lib.CFD_SCHED_PERSISTENT if persistent else 0) | (_lib.CFD_SCHED_SPLIT_X if split_x else 0) |
                 (_lib.CFD_SCHED_XCD if xcd else 0) | (_lib.CFD_SCHED_CONCURRENT if concurrent else 0))
        check(lib().cfd_plan_set_schedule(self._h, N, int(bool(xlines)), partitions, flags))

    set_schedule = cfd_plan_set_schedule

    def cfd_plan_get_schedule(self) -> Dict:
        pers, split, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        cap = 64
        Ns, xs, Ps = (ctypes.c_int * cap)(), (ctypes.c_int * cap)(), (ctypes.c_int * cap)()
        check(lib().cfd_plan_get_schedule(self._h, ctypes.byref(pers), ctypes.byref(split), ctypes.byref(n),
                                          Ns, xs, Ps, cap))
        flags = ctypes.c_int()
        check(lib().cfd_plan_get_flags(self._h, ctypes.byref(flags)))
        return {"persistent": pers.value, "split_x": bool(split.value),
                "concurrent": bool(flags.value & _lib.CFD_SCHED_CONCURRENT), "flags": flags.value,
                "classes": [(Ns[i], xs[i], Ps[i]) for i in range(min(n.value, cap))]}

    get_schedule = cfd_plan_get_schedule

    def cfd_wave_rk_stage(self, u0, src, stage, acc, derivs, a: float, b: float, stream=None, acc_in=None) -> None:
        """stage = u0 + a k (unless stage is None); acc = acc_in + b k (acc_in None: acc itself)."""
        check(lib().cfd_wave_rk_stage(self._h, _dev_ptr(u0), _dev_ptr(src),
                                      _dev_ptr(stage) if stage is not None else None,
                                      _dev_ptr(acc_in) if acc_in is not None else None, _dev_ptr(acc),
                                      _dev_ptr(derivs), float(a), float(b), _stream_ptr(stream)))

    wave_rk_stage = cfd_wave_rk_stage

    def cfd_wave_rk_stage_halo(self, u0, src, stage, acc, derivs, a: float, b: float, bx: int, by: int, bz: int,
                               stream=None, acc_in=None) -> None:
        """wave_rk_stage on a bx x by x bz periodic block lattice, also refreshing the face ghosts of the
        state the next derivative reads (stage, or acc when stage is None)."""
        check(lib().cfd_wave_rk_stage_halo(self._h, _dev_ptr(u0), _dev_ptr(src),
                                           _dev_ptr(stage) if stage is not None else None,
                                           _dev_ptr(acc_in) if acc_in is not None else None, _dev_ptr(acc),
                                           _dev_ptr(derivs), float(a), float(b), int(bx), int(by), int(bz),
                                           _stream_ptr(stream)))

    wave_rk_stage_halo = cfd_wave_rk_stage_halo

    def cfd_wave_rk_stage_fused(self, u0, src, stage, acc, work, a: float, b: float, lattice=None, stream=None,
                                acc_in=None) -> None:
        """The stage with the derivatives folded into the line kernels (two launches; work: a buffer of the
        plan's output size).  stage and acc must not be src or each other.  lattice (bx, by, bz): also
        refresh the face ghosts of the state the next stage reads."""
        bx, by, bz = lattice if lattice is not None else (0, 0, 0)
        check(lib().cfd_wave_rk_stage_fused(self._h, _dev_ptr(u0), _dev_ptr(src),
                                            _dev_ptr(stage) if stage is not None else None,
                                            _dev_ptr(acc_in) if acc_in is not None else None, _dev_ptr(acc),
                                            _dev_ptr(work), float(a), float(b), int(bx), int(by), int(bz),
                                            _stream_ptr(stream)))

    wave_rk_stage_fused = cfd_wave_rk_stage_fused

    def cfd_plan_set_iteration(self, iterations: int, bx: int = 1, by: int = 1, bz: int = 1) -> None:
        """Hybrid closure iteration on a periodic bx x by x bz block lattice (0: plain block closure)."""
        check(lib().cfd_plan_set_iteration(self._h, int(iterations), int(bx), int(by), int(bz)))

    set_iteration = cfd_plan_set_iteration

    def cfd_halo_exchange(self, data, bx: int, by: int, bz: int, stream=None) -> None:
        check(lib().cfd_halo_exchange(self._h, _dev_ptr(data), bx, by, bz, _stream_ptr(stream)))

    halo_exchange = cfd_halo_exchange

    def cfd_plan_set_neighbors(self, nbr) -> None:
        """Face neighbours per block: nbr[b][f] (f = x-, x+, y-, y+, z-, z+), -1 for none."""
        flat = [int(v) for row in nbr for v in row]
        if len(flat) != 6 * self.nblocks:
            raise ValueError("need 6 neighbours per block")
        arr = (ctypes.c_int * len(flat))(*flat)
        check(lib().cfd_plan_set_neighbors(self._h, arr))

    set_neighbors = cfd_plan_set_neighbors

    def cfd_halo_exchange_table(self, data, stream=None) -> None:
        check(lib().cfd_halo_exchange_table(self._h, _dev_ptr(data), _stream_ptr(stream)))

    halo_exchange_table = cfd_halo_exchange_table

    def cfd_plan_set_neighbors_vc(self, nbr) -> None:
        """Vertex-centred tiling: neighbours share their extremal nodes (table as set_neighbors)."""
        flat = [int(v) for row in nbr for v in row]
        if len(flat) != 6 * self.nblocks:
            raise ValueError("need 6 neighbours per block")
        arr = (ctypes.c_int * len(flat))(*flat)
        check(lib().cfd_plan_set_neighbors_vc(self._h, arr))

    set_neighbors_vc = cfd_plan_set_neighbors_vc

    def cfd_shared_node_average(self, data, output: bool = False, stream=None) -> None:
        check(lib().cfd_shared_node_average(self._h, _dev_ptr(data), int(bool(output)), _stream_ptr(stream)))

    shared_node_average = cfd_shared_node_average

    def __del__(self):
        try:
            if self._h:
                lib().cfd_plan_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return CFD_F64
    if t.dtype == torch.float32:
        return CFD_F32
    raise ValueError("float64 or float32 tensors only")


def cfd_axpby(a: float, x, b: float, y, stream=None) -> None:
    """y = a*x + b*y on the GPU."""
    check(lib().cfd_axpby(_dtype_code(y), y.numel(), float(a), _dev_ptr(x), float(b), _dev_ptr(y),
                          _stream_ptr(stream)))


def cfd_apply_block_noalloc(scheme: "Scheme", block: Dict, direction: int, nfields: int, inp, out, field: int = -1,
                            dtype: int = CFD_F64, stream=None) -> None:
    """One operator on every line of one block without a plan and without device allocation."""
    b = _lib.cfd_block()
    b.n = (ctypes.c_int * 3)(*block["n"])
    b.ng = int(block["ng"])
    b.h = (ctypes.c_double * 3)(*block["h"])
    b.boundary = (ctypes.c_int * 3)(*block["boundary"])
    b.in_offset = -1
    b.out_offset = -1
    check(lib().cfd_apply_block_noalloc(scheme._h, ctypes.byref(b), int(direction), int(nfields), int(field),
                                        int(dtype), _dev_ptr(inp), _dev_ptr(out), _stream_ptr(stream)))


def cfd_debug_fail_capture(on: bool = True) -> None:
    """Test hook: the next graph capture takes the eager fallback."""
    lib().cfd_debug_fail_capture(int(bool(on)))


def cfd_debug_fail_alloc(n: int) -> None:
    """Test hook: the library's n-th following device allocation fails (n < 0: off)."""
    lib().cfd_debug_fail_alloc(int(n))


def cfd_xpcy(x, c: float, y, z, stream=None) -> None:
    """z = x + c*y on the GPU."""
    check(lib().cfd_xpcy(_dtype_code(z), z.numel(), _dev_ptr(x), float(c), _dev_ptr(y), _dev_ptr(z),
                         _stream_ptr(stream)))
