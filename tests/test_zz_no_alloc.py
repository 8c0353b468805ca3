"""The allocation-free spectrum entry point against lbw_modes.

lbw_modes_noalloc runs the same spectrum rule as lbw_modes through the
library's fixed device work space, a few probe columns at a time, writing
into caller-owned device buffers.  The same FP64 operations in the same
order: results must be identical bit for bit, on two calls in a row (the
second on a smaller input, so nothing may carry over from the first), one
of them with more probe columns than one pass through the work space holds.
"""
import sys

import numpy as np
import pytest
import torch

import paper_1705_01801_amd as lbw
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(sim, k):
    fh, ph = sim.modes(k)
    fd = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
    pd = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
    sim.modes_noalloc(k, fd, pd)
    torch.cuda.synchronize()
    return fh, ph, fd.cpu().numpy(), pd.cpu().numpy()


def same(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def test_noalloc_modes_match_lbw_modes_on_two_calls():
    # 1: 16 probes over 40,000 rows (nfft 262,144: three columns per pass
    # through the 32 MiB work space, so six passes accumulate the power)
    w = W.workload(1, scale=8)
    say("noalloc 1", w["name"], w["geom"]["n"], "probes", len(w["probes"]))
    g = lbw.Geometry(w["geom"])
    sim = lbw.Simulation(g, w["P0"], w["probes"], t_max=40000)
    sim.step(40000)
    fh, ph, fd, pd = both(sim, 10)
    assert np.isfinite(fh).sum() >= 5
    assert same(fh, fd) and same(ph, pd)
    # 2: a smaller input on the same work space: one probe, 2000 rows
    w2 = W.workload(0)
    say("noalloc 2", w2["name"])
    g2 = lbw.Geometry(w2["geom"])
    sim2 = lbw.Simulation(g2, w2["P0"], w2["probes"], t_max=2000)
    sim2.step(2000)
    fh2, ph2, fd2, pd2 = both(sim2, 6)
    assert np.isfinite(fh2).sum() >= 3
    assert same(fh2, fd2) and same(ph2, pd2)
    # and the first state again, after the small one
    fh3, ph3, fd3, pd3 = both(sim, 10)
    assert same(fh, fd3) and same(ph, pd3)


def test_noalloc_modes_reject_traces_beyond_the_work_space():
    geom = dict(kind="box", dim=2, n=(4, 4), qmin=(0, 0), qmax=(4.0, 4.0), bc_lo=("bounceback", "bounceback"),
                bc_hi=("bounceback", "bounceback"), h_ref=1.0, c=0.4, damp=1.0, params=())
    g = lbw.Geometry(geom)
    P0 = np.random.default_rng(1).uniform(-1, 1, 16)
    sim = lbw.Simulation(g, P0, [0], t_max=131073)
    sim.step(131073)
    fd = torch.zeros(4, dtype=torch.float64, device="cuda")
    pd = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(lbw.LbwError):
        sim.modes_noalloc(4, fd, pd)
    with pytest.raises(lbw.LbwError):
        sim.modes_noalloc(0, fd, pd)
