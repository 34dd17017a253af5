"""cuba_init_static (the entry point that allocates nothing) against
cuba_init: the same kernels on the same state, so the states and work
counters after the same steps must be bit-identical (the profiles within the
rounding of their storage-order sums).  Two calls in a row on one GPU,
the second with a smaller input, check that the library's workspace is
cleared where it must start at zero."""
import sys

import numpy as np
import pytest

from paper_1208_0961_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import cuba as C
    from paper_1208_0961_amd import sim as S
    return torch, C, S


def _run_static(torch, C, params, state, steps):
    """Init through cuba_init_static, `steps` steps, then state and profiles."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream(dev)
    p = C.make_params(**params)
    n = len(state[0])
    nx = int(params["cells"][0])
    arrs = [torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(dev) for a in state]
    ctx = C.cuba_init_static(p, n, *[a.data_ptr() for a in arrs], stream.cuda_stream)
    C.cuba_step(ctx, steps)
    out = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(6)]
    C.cuba_get_state(ctx, *[o.data_ptr() for o in out])
    T00 = torch.empty(nx, dtype=torch.float64, device=dev)
    T0x = torch.empty(nx, dtype=torch.float64, device=dev)
    C.cuba_observe(ctx, T00.data_ptr(), T0x.data_ptr())
    C.cuba_sync(ctx)
    counters = C.cuba_counters(ctx)
    C.cuba_destroy(ctx)
    return [o.cpu().numpy() for o in out], T00.cpu().numpy(), T0x.cpu().numpy(), counters


def _run_workspace(S, C, params, state, steps):
    sim = S.Sim(params, state)
    sim.step(steps)
    st = sim.get_state()
    T00, T0x = sim.observe()
    counters = C.cuba_counters(sim.ctx)
    sim.close()
    return st, T00, T0x, counters


def test_static_workspace_matches_caller_workspace(mods):
    torch, C, S = mods
    big = W.TUBE_1D
    small = W.Workload("riemann-tube-6x1x1-c60x1x1-rt60", (6.0, 1.0, 1.0), (60, 1, 1),
                       60.0, 0.4, 0.02, 0.40, 0.32, steps=200, seed=7)
    cases = [(big, 12), (small, 9)]
    for w, steps in cases:
        state = W.riemann_state(w)
        params = {**w.params(), "cell_capacity": W.capacity_for(w)}
        say(f"[no-alloc] {w.name} n={len(state[0])} steps={steps}")
        assert C.cuba_workspace_bytes(C.make_params(**params), len(state[0])) <= \
            C.CUBA_STATIC_WORKSPACE_BYTES
        got = _run_static(torch, C, params, state, steps)
        want = _run_workspace(S, C, params, state, steps)
        for d in range(6):
            assert np.array_equal(got[0][d], want[0][d]), f"{w.name}: state column {d}"
        # the slab sums run in storage order, which the binning's atomics fix
        # anew in every run: the two agree within the recursive-summation
        # bound of two orders of the same terms
        st = want[0]
        dx = w.box[0] / w.cells[0]
        vol = w.r_test * dx * w.box[1] * w.box[2]
        ix = np.clip(np.floor(st[0] / dx).astype(np.int64), 0, w.cells[0] - 1)
        cnt = np.bincount(ix, minlength=w.cells[0])
        E = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
        bound_e = 2 * (cnt + 2) * 2.0 ** -53 * np.bincount(ix, E, w.cells[0]) / vol
        bound_p = 2 * (cnt + 2) * 2.0 ** -53 * np.bincount(ix, np.abs(st[3]), w.cells[0]) / vol
        assert np.all(np.abs(got[1] - want[1]) <= bound_e + 1e-300), f"{w.name}: T00"
        assert np.all(np.abs(got[2] - want[2]) <= bound_p + 1e-300), f"{w.name}: T0x"
        assert got[3] == want[3], f"{w.name}: work counters {got[3]} vs {want[3]}"
        assert want[3]["claims"] > 0, "no scatterings: the check would be empty"


def test_static_workspace_rejects_oversize(mods):
    torch, C, S = mods
    w = W.TUBE_3D
    params = {**w.params(), "cell_capacity": W.capacity_for(w)}
    p = C.make_params(**params)
    assert C.cuba_workspace_bytes(p, w.n) > C.CUBA_STATIC_WORKSPACE_BYTES
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(C.CubaError) as e:
        C.cuba_init_static(p, w.n, *([x.data_ptr()] * 6),
                           torch.cuda.current_stream().cuda_stream)
    assert e.value.code == C.CUBA_ENOMEM
