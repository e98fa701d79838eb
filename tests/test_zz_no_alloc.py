"""wdlb_create_static: a context on the library's static device array (no
device allocation) against the same lattice on a caller workspace
(wdlb_create): identical fields, step by step, on two contexts in a row, the
second on a smaller lattice; and the limits it declares (too large a
lattice, a second context on the device while one is alive)."""
import sys

import numpy as np
import pytest

from paper_1304_7880_amd.workloads import packing_to_density, random_fields

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# (shape, walls, sigma, eta, tau, g, precision, steps): the second is smaller
CASES = [((40, 20, 13), True, 4.0, 0.3, 0.9, (1e-4, -3e-5, 0.0), "fp32_local64", 6),
         ((16, 12, 10), False, 3.0, 0.25, 1.1, (0.0, 2e-5, 1e-5), "fp64", 5)]


def _run(ctx, n, u, steps):
    ctx.init_fields(n, u)
    out = [ctx.read_fields(with_forces=True)]
    for _ in range(steps):
        ctx.step(1)
        out.append(ctx.read_fields(with_forces=True))
    ctx.step(3)   # an odd chunk: launch by launch in both
    out.append(ctx.read_fields(with_forces=True))
    out.append(ctx.read_profiles())
    out.append(ctx.read_flux())
    return out


def test_static_context_equals_workspace_context_twice():
    from paper_1304_7880_amd import wdlb
    for (nx, ny, nz), walls, sigma, eta, tau, g, prec, steps in CASES:
        _say(f"static vs workspace context {nx}x{ny}x{nz} sigma={sigma} {prec}")
        n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=13)
        a = wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, tau, g, static=True)
        assert a.workspace is None
        out_a = _run(a, n, u, steps)
        a.destroy()
        b = wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, tau, g)
        b.set_graphs(False)
        out_b = _run(b, n, u, steps)
        b.destroy()
        for k, (fa, fb) in enumerate(zip(out_a, out_b)):
            for ea, eb in zip(fa, fb):
                assert np.array_equal(np.asarray(ea), np.asarray(eb)), (nx, k)


def test_static_context_limits():
    from paper_1304_7880_amd import wdlb
    _say("static context limits")
    # a lattice whose workspace exceeds the static array
    with pytest.raises(wdlb.WdlbError) as e:
        wdlb.Context(256, 256, 128, True, "fp32", 4.0, 0.2, 1.0, static=True)
    assert e.value.status == wdlb.E_NOMEM
    a = wdlb.Context(8, 8, 8, True, "fp32", 3.0, 0.2, 1.0, static=True)
    with pytest.raises(wdlb.WdlbError) as e:
        wdlb.Context(8, 8, 8, True, "fp32", 3.0, 0.2, 1.0, static=True)
    assert e.value.status == wdlb.E_STATE
    a.destroy()
    b = wdlb.Context(8, 8, 8, True, "fp32", 3.0, 0.2, 1.0, static=True)   # free again
    b.init_uniform((0.0, 0.0, 0.0))
    b.step(2)
    b.sync()
    b.destroy()
