"""Device memory through the registered allocator (twa_set_allocator): a
solver's, a batch's and twa_backward's buffers come from the callbacks,
go back through them at destroy, and the results do not depend on where
the memory came from."""
import gc

import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu


class _Counting:
    """torch's caching allocator behind callbacks that keep a ledger."""

    def __init__(self):
        import torch
        import paper_1311_4527_amd.twa as T
        self.live = {}
        self.calls = 0

        def alloc(n, dev, stream, ctx):
            self.calls += 1
            p = torch.cuda.caching_allocator_alloc(int(n), device=int(dev), stream=int(stream or 0))
            self.live[p] = int(n)
            return p

        def free(p, n, dev, stream, ctx):
            assert self.live.pop(int(p)) == int(n)
            torch.cuda.caching_allocator_delete(int(p))

        self.a = T._ALLOC_FN(alloc)
        self.f = T._FREE_FN(free)
        assert T.load_library().twa_set_allocator(self.a, self.f, None) == 0

    def restore(self):
        import paper_1311_4527_amd.twa as T
        T.twa_set_allocator(True)


def test_solver_and_backward_buffers_come_from_the_callbacks():
    import torch
    import paper_1311_4527_amd.twa as T
    inst = I.conf_adjoint(3, p=8)
    ref = T.Solver.from_instance(inst, flags=T.TWA_F_TAPE)
    ref.twa_iterate(40)
    z_ref = ref.twa_get_trajectories()
    g_ref = ref.twa_backward(torch.ones_like(z_ref))
    C = _Counting()
    try:
        S = T.Solver.from_instance(inst, flags=T.TWA_F_TAPE)
        n_create = C.calls
        assert n_create > 0 and len(C.live) == n_create
        S.twa_iterate(40)
        z = S.twa_get_trajectories()
        assert torch.equal(z, z_ref)
        g = S.twa_backward(torch.ones_like(z))
        assert C.calls > n_create        # the adjoint's buffers
        # (the adjoint sums cotangents with float atomics: equal up to the
        # rounding of their order)
        for a, b in zip(g, g_ref):
            scale = float(b.abs().max())
            assert torch.allclose(a, b, rtol=1e-4, atol=1e-4 * scale), float((a - b).abs().max())
        S.close()
        assert not C.live                # everything went back through release
    finally:
        C.restore()
    ref.close()


def test_batch_buffers_come_from_the_callbacks():
    import torch
    import paper_1311_4527_amd.twa as T
    insts = I.conf_batch(4, base_seed=3, p_range=(4, 20))
    C = _Counting()
    try:
        B = T.Batch(insts)
        assert C.live
        B.twa_batch_iterate(10)
        z = [B.twa_batch_get_trajectories(i) for i in range(len(insts))]
        B.close()
        assert not C.live
    finally:
        C.restore()
    for i, inst in enumerate(insts):
        S = T.Solver.from_instance(inst)
        S.twa_iterate(10)
        assert torch.equal(S.twa_get_trajectories(), z[i])
        S.close()


def test_default_allocator_is_torch_and_a_failed_alloc_is_nomem():
    import torch
    import paper_1311_4527_amd.twa as T
    inst = I.random_box(64, 0.01, 8, seed=2, C=1 / 512)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    S = T.Solver.from_instance(inst)
    assert torch.cuda.memory_allocated() > before     # the solver's buffers are torch's
    S.close()
    del S      # and the wrapper's own input tensors
    gc.collect()
    assert torch.cuda.memory_allocated() == before
    fail_a = T._ALLOC_FN(lambda n, d, s, c: None)
    fail_f = T._FREE_FN(lambda p, n, d, s, c: None)
    assert T.load_library().twa_set_allocator(fail_a, fail_f, None) == 0
    try:
        with pytest.raises(T.TWAError) as e:
            T.Solver.from_instance(inst)
        assert e.value.status == T.TWA_E_NOMEM
    finally:
        T.twa_set_allocator(True)
