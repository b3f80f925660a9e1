"""Host-side argument checks of the C ABI that need a plan (hence a GPU): overlapping inputs
and outputs are rejected with FX_EINVAL before anything is launched, pass tensors beyond
32-bit indexing with FX_EUNSUPPORTED before any pass runs, and the stacked calls agree with
the single-field calls field by field."""

import ctypes

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


def _L():
    from paper_1602_03395_amd import _lib as L
    return L


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def Poff(t, elems):
    return ctypes.c_void_p(t.data_ptr() + elems * t.element_size())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_overlapping_pointers_are_rejected(fx, dtype):
    L = _L()
    shape, lam = (12, 16), (3, 4)
    plan = fx.Plan(shape, (1.0, 1.0), 1.0, 5.0, lam, dtype=dtype)
    h = plan.handle
    n = shape[0] * shape[1]
    big = torch.zeros(4 * n, dtype=dtype, device="cuda")
    rbig = torch.zeros(4 * n, dtype=fx.real_dtype(dtype), device="cuda")
    s = stream()
    # output == input, output inside input, two outputs sharing memory
    assert L.lib.fx_expand(h, P(big), P(big), None, s) == L.FX_EINVAL
    assert b"overlap" in L.lib.fx_last_error()
    assert L.lib.fx_expand(h, P(big), Poff(big, n // 2), None, s) == L.FX_EINVAL
    assert L.lib.fx_expand(h, P(big), Poff(big, n), Poff(big, n), s) == L.FX_EINVAL
    assert L.lib.fx_expand_range(h, P(big), P(big), 0, 3, 0, s) == L.FX_EINVAL
    assert L.lib.fx_expand_adjoint(h, P(big), Poff(big, n - 1), s) == L.FX_EINVAL
    assert L.lib.fx_density(h, P(big), P(big), s) == L.FX_EINVAL
    assert L.lib.fx_density_adjoint(h, P(big), P(rbig), P(big), s) == L.FX_EINVAL
    assert L.lib.fx_expand_pair(h, P(big), Poff(big, n), Poff(big, n), None, None, s) == L.FX_EINVAL
    assert L.lib.fx_expand_pair(h, P(big), Poff(big, n), Poff(big, 2 * n), Poff(big, 2 * n), None, s) == L.FX_EINVAL
    assert L.lib.fx_far_field(h, P(big), P(big), None, s) == L.FX_EINVAL
    assert L.lib.fx_brute_force(h, P(big), Poff(big, 1), None, s) == L.FX_EINVAL
    assert L.lib.fx_expand_many(h, 2, P(big), Poff(big, n), None, s) == L.FX_EINVAL
    assert L.lib.fx_density_adjoint_many(h, 2, P(big), P(rbig), Poff(big, n), s) == L.FX_EINVAL
    # adjacent, disjoint buffers are accepted
    assert L.lib.fx_expand(h, P(big), Poff(big, n), Poff(rbig, 0), s) == L.FX_OK
    torch.cuda.synchronize()


def test_batch_rejects_overlapping_outputs(fx):
    shapes = [(8, 12), (8, 12), (6, 10)]
    psis = [torch.from_numpy(workloads.random_field(s, i).astype(np.complex64)).cuda() for i, s in enumerate(shapes)]
    b = fx.Batch([dict(shape=s, dx=(1.0, 1.0), lam=(2, 3), t=3.0) for s in shapes], dtype=torch.complex64)
    outs = [torch.empty_like(x) for x in psis]
    rhos = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for x in psis]
    with pytest.raises(ValueError, match="overlap"):
        b.run(psis, psi_outs=[outs[0], outs[0], outs[2]], rho_outs=rhos)
    with pytest.raises(ValueError, match="overlap"):
        b.run(psis, psi_outs=[psis[1], outs[1], outs[2]], rho_outs=rhos)
    # the same input for several realizations is fine
    b.run([psis[0], psis[0], psis[2]], psi_outs=outs, rho_outs=rhos)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


def test_pass_tensor_beyond_32bit_indexing_is_rejected_before_launch(fx):
    # 3-D field of 2^30 points whose middle pass tensor (lam_y * Mz * Py * Px) exceeds 2^31 elements
    # even with the outermost magnification index blocked to 1: rejected before any pass is enqueued
    L = _L()
    shape, lam = (64, 4096, 4096), (1, 3, 1)
    plan = fx.Plan(shape, (1.0, 1.0, 1.0), 1.0, 1.0, lam, dtype=torch.complex64)
    n = 64 * 4096 * 4096
    x = torch.zeros(n, dtype=torch.complex64, device="cuda")
    y = torch.empty(n, dtype=torch.complex64, device="cuda")
    st = L.lib.fx_expand(plan.handle, P(x), P(y), None, stream())
    assert st == L.FX_EUNSUPPORTED
    assert b"2^31" in L.lib.fx_last_error()
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 1e-6)])
def test_stacked_calls_equal_single_calls(fx, dtype, tol):
    shape, lam, dx, t = (24, 40), (4, 8), (1.0, 0.8), 6.0
    count = 5
    fields = np.stack([workloads.random_field(shape, 50 + i) for i in range(count)])
    x = torch.from_numpy(fields.astype(np.complex64 if dtype == torch.complex64 else np.complex128)).cuda()
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=dtype)
    out, rho = plan.expand_many(x)
    g_rho = torch.rand(rho.shape, dtype=rho.dtype, device="cuda")
    grad = plan.density_adjoint_many(out, g_rho)
    torch.cuda.synchronize()
    for b in range(count):
        o1, r1 = plan.expand(x[b].contiguous())
        g1 = plan.density_adjoint(o1, g_rho[b].contiguous())
        torch.cuda.synchronize()
        assert torch.allclose(out[b], o1, rtol=0, atol=tol * o1.abs().max().item())
        assert torch.allclose(grad[b], g1, rtol=0, atol=tol * g1.abs().max().item())
        ref = oracle.expand(x[b].cpu().numpy().astype(np.complex128), dx, 1.0, t, lam)
        assert np.linalg.norm(out[b].cpu().numpy() - ref) <= 10 * tol * np.linalg.norm(ref)


def test_stacked_calls_chunk_under_a_small_caller_workspace(fx):
    # a caller workspace sized for one field forces one field per chunk
    shape, lam, dx, t = (16, 20), (2, 5), (1.0, 1.0), 4.0
    count = 3
    x = torch.from_numpy(np.stack([workloads.random_field(shape, 70 + i) for i in range(count)])).cuda()
    plan = fx.Plan(shape, dx, 1.0, t, lam, dtype=torch.complex128)
    plan.use_torch_workspace()
    out, _ = plan.expand_many(x)
    torch.cuda.synchronize()
    for b in range(count):
        ref = oracle.expand(x[b].cpu().numpy(), dx, 1.0, t, lam)
        assert np.linalg.norm(out[b].cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
