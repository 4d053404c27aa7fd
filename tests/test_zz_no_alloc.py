"""The allocation-free reduction (pflbm_reduce_static, partial sums in the
library's static device array) against pflbm_reduce (partial sums in the
context's workspace), through the C ABI: bitwise the same sums on two calls in
a row, the second on a smaller lattice, so the first call's partials left in
the shared array must not leak into the second."""
import ctypes as C

import pytest

import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu


def _both(sim):
    from paper_2206_11637_amd import _lib
    a = (C.c_double * 5)()
    b = (C.c_double * 5)()
    _lib.check(sim.lib.pflbm_reduce(sim.ctx, a), sim.ctx, "pflbm_reduce")
    _lib.check(sim.lib.pflbm_reduce_static(sim.ctx, b), sim.ctx, "pflbm_reduce_static")
    return list(a), list(b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_reduction_matches_the_workspace_reduction(precision):
    from paper_2206_11637_amd.sim import from_workload
    for shape, steps in (((96, 40, 24), 7), ((37, 11, 6), 3)):
        say(f"case: reduce_static {precision} {shape} after {steps} steps")
        wl = W.random_state(*shape, periodic=(True, False, True), solid_fraction=0.05, seed=3)
        sim = from_workload(wl, precision=precision)
        sim.step(steps)
        ws, st = _both(sim)
        say(f"  workspace {ws}\n  static    {st}")
        assert ws == st
        # and again on the same state: the array keeps the last call's contents
        ws2, st2 = _both(sim)
        assert ws2 == ws and st2 == st
        del sim
