"""Classical RK4 for the first-order wave system on the GPU (workload driver).

State: five fields (phi, Pi, psi_x, psi_y, psi_z) on mesh blocks.  Each stage
is either one batched derivative apply of the plan (D_x, D_y, D_z of Pi and
D_i psi_i) followed by one stage kernel (cfd_wave_rk_stage; on block lattices
cfd_wave_rk_stage_halo, which also refreshes the face ghosts), or, fused
(cfd_wave_rk_stage_fused), two line-kernel launches whose epilogues perform
the stage update, so that only D_x psi_x and D_y psi_y pass through memory.
The fused stages alternate between two stage buffers.  A whole step can be
captured in one HIP graph.
"""
from __future__ import annotations

from typing import Dict, List, Optional

from . import CFD_F32, CFD_F64, Plan, Scheme


def wave_ops(scheme: Scheme):
    """The six operators the stage kernel expects, in its order."""
    return [(scheme, 0, 1), (scheme, 1, 1), (scheme, 2, 1), (scheme, 0, 2), (scheme, 1, 3), (scheme, 2, 4)]


class WaveRK4:
    def __init__(self, blocks: List[Dict], scheme: Scheme, dt: float, dtype: int = CFD_F64,
                 lattice: Optional[tuple] = None, fused: bool = False):
        import torch
        self.plan = Plan(blocks, 5, wave_ops(scheme), dtype=dtype)
        self.dt = float(dt)
        self.lattice = lattice
        self.fused = fused
        nin, nout = self.plan.sizes()
        tdt = torch.float64 if dtype == CFD_F64 else torch.float32
        self.u = torch.zeros(nin, dtype=tdt, device="cuda")
        self.stage = torch.zeros_like(self.u)
        self.stage2 = torch.zeros_like(self.u) if fused else None
        self.acc = torch.zeros_like(self.u)
        self.d = torch.zeros(nout, dtype=tdt, device="cuda")
        self.graph = None

    def load(self, host_state):
        import torch
        self.u.copy_(torch.as_tensor(host_state, dtype=self.u.dtype))
        self._halo(self.u)
        self.stage.copy_(self.u)
        if self.stage2 is not None:
            self.stage2.copy_(self.u)

    def _halo(self, buf):
        if self.lattice is not None:
            self.plan.halo_exchange(buf, *self.lattice)

    def step(self):
        """u <- RK4 step of size dt (the first stage reads acc from u, the last writes u).  On a block
        lattice the stage kernel also refreshes the ghosts of the state the next stage reads."""
        dt = self.dt
        src = self.u
        stages = ((dt / 2, dt / 6), (dt / 2, dt / 3), (dt, dt / 3), (None, dt / 6))
        if self.fused:
            bufs = (self.stage, self.stage2, self.stage, None)
            for i, (a, b) in enumerate(stages):
                last = i == len(stages) - 1
                self.plan.wave_rk_stage_fused(self.u, src, bufs[i], self.u if last else self.acc, self.d,
                                              0.0 if a is None else a, b, lattice=self.lattice,
                                              acc_in=self.u if i == 0 else self.acc)
                src = bufs[i]
            return
        for i, (a, b) in enumerate(stages):
            self.plan.apply(src, self.d)
            last = i == len(stages) - 1
            args = (self.u, src, None if last else self.stage, self.u if last else self.acc, self.d,
                    0.0 if a is None else a, b)
            acc_in = self.u if i == 0 else self.acc
            if self.lattice is not None:
                self.plan.wave_rk_stage_halo(*args, *self.lattice, acc_in=acc_in)
            else:
                self.plan.wave_rk_stage(*args, acc_in=acc_in)
            src = self.stage

    def capture(self):
        """Capture one step in a HIP graph (torch.cuda.CUDAGraph); run() then replays it."""
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.step()          # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step()

    def run(self, nsteps: int):
        for _ in range(nsteps):
            if self.graph is not None:
                self.graph.replay()
            else:
                self.step()
