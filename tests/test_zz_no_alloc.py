"""twa_backward_noalloc (the adjoint for callers that cannot allocate: every
buffer from the library's static scratch) against twa_backward, through the
C ABI: two calls in a row on one device, the second with a smaller problem,
so the second runs on scratch the first left filled."""
import numpy as np
import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu


def _check(inst, K, seed):
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    S.twa_iterate(K)
    v = torch.from_numpy(np.random.default_rng(seed).normal(size=inst.z0.shape).astype(np.float32)).cuda()
    z_before = S.twa_get_trajectories().clone()
    outs = [torch.full((inst.p, 2), float("nan"), device="cuda"), torch.full((inst.p, 2), float("nan"), device="cuda"),
            torch.full((inst.p,), float("nan"), device="cuda"), torch.full(inst.z0.shape, float("nan"), device="cuda",
                                                                           dtype=torch.float32)]
    S.twa_backward_noalloc(v, *outs)
    torch.cuda.synchronize()
    got = [t.cpu().numpy().astype(np.float64) for t in outs]
    want = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(v)]
    for name, g, w in zip(("dx0", "dxT", "dr", "dz0"), got, want):
        assert np.all(np.isfinite(g)), name
        # the same kernels on the same recomputed decisions; the reverse steps
        # sum node cotangents with float atomics, whose order differs from run
        # to run and compounds over 500 steps (observed up to ~4e-6 of the
        # largest entry), so the bar is 1e-4 of it: ten times tighter than the
        # adjoint's 1e-3 against the reference
        scale = max(np.abs(w).max(), 1e-30)
        assert np.allclose(g, w, rtol=1e-4, atol=1e-4 * scale), (name, np.abs(g - w).max(), scale)
    # the solver's forward state is untouched, and the run continues bitwise
    assert torch.equal(S.twa_get_trajectories(), z_before)
    R = Solver.from_instance(inst, flags=TWA_F_TAPE)
    R.twa_iterate(K + 7)
    S.twa_iterate(7)
    assert torch.equal(S.twa_get_trajectories(), R.twa_get_trajectories())
    print(f"noalloc {inst.name} K={K}: max |dr| {np.abs(want[2]).max():.3e}", flush=True)


def test_noalloc_backward_matches_backward_twice():
    # first the 256-agent swap for 500 iterations, then a smaller problem:
    # its 8-agent sub-instance for 40 iterations, on scratch the first filled
    _check(I.conf_adjoint(7), 500, 0)
    _check(I.sub_instance(I.conf_adjoint(7), np.arange(0, 256, 32)), 40, 1)


def test_noalloc_backward_rejects_what_does_not_fit():
    """A run whose buffers exceed the scratch is refused with TWA_E_NOMEM
    (and leaves the solver usable); twa_backward has no such limit."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWAError, TWA_E_NOMEM, TWA_F_TAPE
    inst = I.random_box(1100, 0.004, 8, min_sep=0.01, seed=5, alpha=0.1, C=1 / 8800)
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    S.twa_iterate(4)
    v = torch.ones(inst.z0.shape, device="cuda")
    outs = [torch.empty((inst.p, 2), device="cuda"), torch.empty((inst.p, 2), device="cuda"),
            torch.empty((inst.p,), device="cuda"), None]
    with pytest.raises(TWAError) as e:
        S.twa_backward_noalloc(v, *outs)
    assert e.value.status == TWA_E_NOMEM
    S.twa_iterate(1)
    S.twa_check_finite()
