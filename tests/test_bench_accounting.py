"""The byte accounting behind bench.py's roofline figure (CPU only)."""
import numpy as np

import bench
import synth


def _wl(boundary):
    blk = synth.Block((4, 5, 6), 2, (0.1, 0.1, 0.1), boundary, (0.0, 0.0, 0.0))
    return synth.Workload("tiny", [blk], 3, np.zeros(1), [0])


def test_algorithmic_bytes_hand_count():
    """3 fields of a 4x5x6 block with 2 ghost layers, operators along x and z: every interior value and the
    x and z ghost faces read once (no edges or corners), every output written once."""
    ops = [("(1)Q1_3[1]", 0), ("(2)Q1_3[1]", 2)]
    alg, rd, wr = bench.algorithmic_bytes(_wl((synth.CLOSURE,) * 3), ops, 8)
    n3 = 4 * 5 * 6
    reads = 3 * (n3 + 2 * 2 * (5 * 6) + 2 * 2 * (4 * 5))
    writes = 2 * 3 * n3
    assert (rd, wr, alg) == (8 * reads, 8 * writes, 8 * (reads + writes))


def test_periodic_directions_read_no_ghosts():
    ops = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 2)]
    _, rd, _ = bench.algorithmic_bytes(_wl((synth.PERIODIC, synth.CLOSURE, synth.CLOSURE)), ops, 4)
    assert rd == 4 * 3 * (4 * 5 * 6 + 2 * 2 * (4 * 5))


def test_batch64_totals():
    """The per-step figures the roofline quotes for batch64 in FP64."""
    wl = synth.batch64()
    alg, rd, wr = bench.algorithmic_bytes(wl, bench.OPS_PENTA, 8)
    evals = sum(len(bench.OPS_PENTA) * wl.nfields * int(np.prod(b.n)) for b in wl.blocks)
    assert (alg, rd, wr, evals) == (2465261568, 615081984, 1850179584, 231272448)
