"""Parity of the HIP path (through the C ABI) with the CPU oracle on the same seeded inputs.

Bars (written per result):
  * plain FP64 (complex128):            relative L2 error of Psibar and of rho <= 1e-12
  * FP32 data + FP64-built phase tables: relative L2 error of rho <= 1e-5
    (the oracle consumes the complex64 input upcast exactly, so input rounding
    is not charged to the method).
"""

import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_RHO = 1e-5


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_03395_amd as m
    return m


CASES = [
    # shape, lam, dx, t, m_over_hbar, abar shift (units of dx)
    ((64,), (5,), (0.5,), 3.0, 1.0, 0.0),
    ((96,), (8,), (1.0,), 40.0, 1.0, 0.25),
    ((45,), (4,), (1.0,), 20.0, 1.3, 0.3),
    ((7,), (3,), (0.7,), 2.0, 1.0, -0.4),
    ((1024,), (10,), (0.1,), 50.0, 1.0, 0.0),
    ((48, 40), (3, 4), (1.0, 0.8), 30.0, 1.0, 0.37),
    ((33, 20), (2, 5), (1.0, 1.0), 12.0, 2.0, 0.0),
    ((64, 64), (8, 16), (1.0, 1.0), 200.0, 1.0, 0.0),
    ((17, 12), (1, 3), (1.0, 1.0), 5.0, 1.0, 0.5),
    ((12, 10, 16), (2, 3, 4), (1.0, 1.0, 1.0), 9.0, 1.0, 0.2),
    ((9, 8, 20), (3, 2, 5), (1.0, 0.5, 1.0), 6.0, 1.0, 0.0),
    ((5, 1, 24), (2, 1, 3), (1.0, 1.0, 1.0), 4.0, 1.0, 0.0),
    ((1, 8), (3, 2), (1.0, 1.0), 3.0, 1.0, 0.0),
    ((16, 384), (2, 3), (1.0, 1.0), 50.0, 1.0, 0.0),
    ((3,), (1,), (1.0,), 1.0, 1.0, 0.0),
    ((12, 24, 48), (2, 3, 4), (1.0, 1.0, 1.0), 7.0, 1.0, 0.1),
    ((96,), (6,), (1.0,), 30.0, 1.0, 0.0),
    # register-form passes: pruned lengths 3, 6, 12, 16, 2, 1 with 2..64 lanes per line
    ((24,), (8,), (1.0,), 10.0, 1.0, 0.0),
    ((32, 48), (2, 8), (1.0, 1.0), 20.0, 1.0, 0.3),
    ((64, 32), (32, 64), (1.0, 1.0), 300.0, 1.0, 0.0),
    ((1024,), (64,), (1.0,), 400.0, 1.0, 0.0),
    ((8, 96), (4, 8), (1.0, 0.5), 25.0, 1.0, 0.2),
    ((40, 12, 48), (8, 2, 4), (1.0, 1.0, 1.0), 15.0, 1.0, 0.0),
    ((64, 64), (2, 6), (1.0, 1.0), 40.0, 1.0, 0.1),     # 32 points per lane (FP32 register form)
]


def _run(fx, psi_np, dtype, lam, dx, t, moh, a, abar, schedule):
    psi = torch.from_numpy(psi_np.astype(np.complex128 if dtype == torch.complex128 else np.complex64)).cuda()
    plan = fx.get_plan(psi.shape, dx, moh, t, lam, a, abar, dtype, schedule)
    out, rho = plan.expand(psi)
    torch.cuda.synchronize()
    return psi, out.cpu().numpy(), rho.cpu().numpy()


@pytest.mark.parametrize("schedule", ["paper", "axis_factorised"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_cases_fp64(fx, case, schedule):
    shape, lam, dx, t, moh, shift = CASES[case]
    say("case", shape, lam, schedule, "fp64")
    psi_np = workloads.random_field(shape, 100 + case)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    ref = oracle.expand(psi_np, dx, moh, t, lam, a, abar)
    _, out, rho = _run(fx, psi_np, torch.complex128, lam, dx, t, moh, list(a), list(abar), schedule)
    e_psi = rel(out, ref)
    e_rho = rel(rho, oracle.density(ref))
    say(f"  rel L2 psi {e_psi:.2e}  rho {e_rho:.2e}")
    assert e_psi <= TOL64 and e_rho <= TOL64


@pytest.mark.parametrize("schedule", ["paper", "axis_factorised"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_small_cases_fp32_phase64(fx, case, schedule):
    shape, lam, dx, t, moh, shift = CASES[case]
    say("case", shape, lam, schedule, "fp32")
    psi_np = workloads.random_field(shape, 200 + case).astype(np.complex64)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    ref = oracle.expand(psi_np.astype(np.complex128), dx, moh, t, lam, a, abar)
    _, out, rho = _run(fx, psi_np, torch.complex64, lam, dx, t, moh, list(a), list(abar), schedule)
    e_rho = rel(rho, oracle.density(ref))
    e_psi = rel(out, ref)
    say(f"  rel L2 rho {e_rho:.2e}  psi {e_psi:.2e}")
    assert e_rho <= TOL32_RHO


def test_expand_range_partitions_sum_to_full(fx):
    shape, lam, dx, t = (10, 12, 16), (2, 3, 4), (1.0, 1.0, 1.0), 7.0
    say("expand_range", shape, lam)
    psi_np = workloads.random_field(shape, 7)
    psi = torch.from_numpy(psi_np).cuda()
    plan = fx.get_plan(shape, dx, 1.0, t, lam)
    Q = plan.num_terms()
    assert Q == 24
    full, _ = plan.expand(psi)
    acc = torch.zeros_like(psi)
    cuts = [0, 1, 5, 6, 11, 12, 13, 23, 24]
    for b, e in zip(cuts[:-1], cuts[1:]):
        plan.expand_range(psi, acc, b, e, accumulate=True)
    torch.cuda.synchronize()
    assert rel(acc.cpu().numpy(), full.cpu().numpy()) <= 1e-13
    part = torch.empty_like(psi)
    plan.expand_range(psi, part, 0, 13, accumulate=False)
    plan.expand_range(psi, part, 13, 24, accumulate=True)
    assert rel(part.cpu().numpy(), full.cpu().numpy()) <= 1e-13
    ref = oracle.expand(psi_np, dx, 1.0, t, lam)
    assert rel(acc.cpu().numpy(), ref) <= TOL64


@pytest.mark.parametrize("schedule", ["paper", "axis_factorised"])
@pytest.mark.parametrize("shape,lam", [((40,), (6,)), ((24, 18), (3, 4)), ((8, 9, 12), (2, 3, 2))])
def test_adjoint_matches_oracle(fx, shape, lam, schedule):
    say("adjoint", shape, lam, schedule)
    dx = tuple(1.0 for _ in shape)
    y_np = workloads.random_field(shape, 31)
    x_np = workloads.random_field(shape, 32)
    plan = fx.get_plan(shape, dx, 1.0, 5.0, lam, schedule=schedule)
    y = torch.from_numpy(y_np).cuda()
    x = torch.from_numpy(x_np).cuda()
    g = plan.expand_adjoint(y).cpu().numpy()
    ref = oracle.expand_adjoint(y_np, dx, 1.0, 5.0, lam)
    assert rel(g, ref) <= TOL64
    ux, _ = plan.expand(x)
    lhs = np.vdot(ux.cpu().numpy(), y_np)
    rhs = np.vdot(x_np, g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# the fused transform + structured accumulate pass (g = 8..64, power-of-two P <= g), on the
# contiguous axis of a 1-D field and on strided axes
@pytest.mark.parametrize("shape,lam,dtype", [
    ((512,), (32,), torch.complex64),
    ((64, 256), (32, 4), torch.complex128),
    ((64, 256), (32, 4), torch.complex64),
    ((256, 128), (16, 8), torch.complex64),
    ((32, 24, 16), (8, 3, 2), torch.complex128),
    ((128, 16), (64, 2), torch.complex128),
    ((128, 16), (64, 2), torch.complex64),
])
def test_structured_ea_matches_oracle(fx, shape, lam, dtype, monkeypatch):
    import json
    monkeypatch.setenv("FX_EAS", "1")  # wherever it applies (by default only for P >= 8)
    monkeypatch.setenv("FX_NO_EAW", "1")  # g = 8 would otherwise take the one-wave-per-tile kernel
    say("structured EA", shape, lam, dtype)
    dx = tuple(0.9 for _ in shape)
    psi_np = workloads.random_field(shape, 81)
    plan = fx.Plan(shape, dx, 1.0, 13.0, lam, dtype=dtype)  # not cached: the switch is read at creation
    assert any(p.get("eas") for p in json.loads(plan.describe())["passes"])
    out, rho = plan.expand(torch.from_numpy(psi_np).to(dtype).cuda())
    ref = oracle.expand(psi_np, dx, 1.0, 13.0, lam)
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= TOL64
    assert rel(rho.cpu().numpy(), oracle.density(ref)) <= (TOL64 if dtype == torch.complex128 else TOL32_RHO)


# g = gcd(lam, M) of 16, 32 and 64: the adjoint accumulate with g / 8 lanes per group
@pytest.mark.parametrize("shape,lam", [((64,), (16,)), ((24, 64), (3, 32)), ((128,), (64,)), ((48, 40), (16, 2)),
                                       ((256,), (16,)), ((64, 64), (8, 8))])
def test_adjoint_lane_groups_match_oracle(fx, shape, lam):
    say("adjoint lanes", shape, lam)
    dx = tuple(1.0 for _ in shape)
    y_np = workloads.random_field(shape, 33)
    plan = fx.get_plan(shape, dx, 1.0, 7.0, lam)
    g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 7.0, lam)) <= TOL64


@pytest.mark.parametrize("shape,lam", [((48, 64), (4, 32)), ((512,), (32,)), ((64, 128), (8, 8))])
def test_adjoint_fp32_form_matches_oracle(fx, shape, lam):
    dx = (1.0,) * len(shape)
    say("adjoint fp32", shape, lam)
    y_np = workloads.random_field(shape, 34)
    plan = fx.get_plan(shape, dx, 1.0, 9.0, lam, dtype=torch.complex64)
    g = plan.expand_adjoint(torch.from_numpy(y_np).to(torch.complex64).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 9.0, lam)) <= TOL32_RHO


EH2_CASES = [
    # shape, lam, dtype: adjoint passes along power-of-two axes of 256..2048 points whose pruned
    # length exceeds the register forms take the compile-time kernel (k_EH2)
    ((256,), (5,), torch.complex128),            # g = 1, P = 256, 1-D
    ((2048,), (3,), torch.complex128),           # one term per round
    ((8, 512), (3, 6), torch.complex128),        # g = 2, P = 256, contiguous lines
    ((256, 64), (20, 4), torch.complex128),      # strided lines (S = 16) after the split AH
    ((1024, 16), (4, 2), torch.complex128),      # P = 256 of M = 1024, strided
    ((256, 256), (20, 20), torch.complex128),    # one field of the gradient workload
    ((256, 256), (20, 20), torch.complex64),
]


@pytest.mark.parametrize("case", range(len(EH2_CASES)))
def test_adjoint_power_of_two_kernel_matches_oracle(fx, case, monkeypatch):
    monkeypatch.setenv("FX_ERW", "0")  # P = 64 with g = 4 would otherwise take the lane-layout adjoint
    shape, lam, dtype = EH2_CASES[case]
    dx = (1.0,) * len(shape)
    say("adjoint eh2", shape, lam, dtype)
    y_np = workloads.random_field(shape, 990 + case)
    if dtype == torch.complex64:
        y_np = y_np.astype(np.complex64).astype(np.complex128)
    plan = fx.Plan(shape, dx, 1.0, 23.0, lam, dtype=dtype)
    import json
    assert any(o.get("eh2") for o in json.loads(plan.describe())["adjoint_passes"])
    g = plan.expand_adjoint(torch.from_numpy(y_np).to(dtype).cuda()).cpu().numpy()
    ref = oracle.expand_adjoint(y_np, dx, 1.0, 23.0, lam)
    assert rel(g, ref) <= (TOL64 if dtype == torch.complex128 else TOL32_RHO)


def test_adjoint_power_of_two_kernel_blocked(fx, monkeypatch):
    # a tiny workspace splits the outer magnification index into blocks: the compile-time adjoint
    # pass then starts at a term index qb > 0 and accumulates into the output
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    monkeypatch.setenv("FX_ERW", "0")
    shape, lam, dx = (256, 256), (20, 20), (1.0, 1.0)
    say("adjoint eh2 blocked", shape, lam)
    y_np = workloads.random_field(shape, 999)
    plan = fx.Plan(shape, dx, 1.0, 23.0, lam)
    import json
    d = json.loads(plan.describe())
    assert d["outer_block"] < 20 and any(o.get("eh2") for o in d["adjoint_passes"])
    g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 23.0, lam)) <= TOL64


MAX_AXIS_CASES = [
    # the longest supported axes: 4096 points in the FP32 form; in plain FP64 the fused pass's
    # LDS ((4 M + 256) 16 bytes <= 160 KiB) allows M <= 2496 (here 2496 = 2^6 3 13, runtime radices)
    ((4096,), (3,), torch.complex64),
    ((48, 4096), (2, 4), torch.complex64),
    ((2496,), (3,), torch.complex128),
    ((2048,), (5,), torch.complex128),
]


def test_fp64_axis_beyond_lds_is_rejected(fx):
    from paper_1602_03395_amd._lib import FxError
    with pytest.raises(FxError) as e:
        fx.Plan((4096,), (1.0,), 1.0, 50.0, (3,), dtype=torch.complex128)
    assert "axis too long" in str(e.value)


@pytest.mark.parametrize("case", range(len(MAX_AXIS_CASES)))
def test_maximum_axis_length_matches_oracle(fx, case):
    shape, lam, dtype = MAX_AXIS_CASES[case]
    dx = (1.0,) * len(shape)
    say("maximum axis", shape, lam, dtype)
    psi_np = workloads.random_field(shape, 1000 + case)
    if dtype == torch.complex64:
        psi_np = psi_np.astype(np.complex64).astype(np.complex128)
    ref = oracle.expand(psi_np, dx, 1.0, 50.0, lam)
    plan = fx.Plan(shape, dx, 1.0, 50.0, lam, dtype=dtype)
    out, rho = plan.expand(torch.from_numpy(psi_np).to(dtype).cuda())
    torch.cuda.synchronize()
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= TOL64
        assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL64
        if len(shape) == 1:
            y_np = workloads.random_field(shape, 1010 + case)
            g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
            assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 50.0, lam)) <= TOL64
    else:
        assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL32_RHO


def test_adjoint_blocked_outer_axis_matches_oracle(fx, monkeypatch):
    # a tiny workspace splits the outer magnification index into blocks whose first index is not
    # a multiple of g = 32: every block's adjoint accumulate carries the phase of its offset
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    shape, lam, dx = (128, 512), (4, 32), (1.0, 1.0)
    say("adjoint blocked", shape, lam)
    y_np = workloads.random_field(shape, 35)
    plan = fx.Plan(shape, dx, 1.0, 11.0, lam)
    import json
    assert json.loads(plan.describe())["outer_block"] < 32
    g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 11.0, lam)) <= TOL64


def test_autograd_gradient_matches_oracle_and_fd(fx):
    shape, lam, dx, t = (16, 20), (3, 2), (1.0, 1.0), 6.0
    say("autograd", shape, lam)
    psi_np = workloads.random_field(shape, 41)
    tau = np.abs(workloads.random_field(shape, 42)) ** 2 * 0.05
    psi = torch.from_numpy(psi_np).cuda().requires_grad_(True)
    tau_t = torch.from_numpy(tau).cuda()
    rho = fx.expand_density(psi, dx, 1.0, t, lam)
    loss = ((rho - tau_t) ** 2).sum()
    loss.backward()
    g = psi.grad.cpu().numpy()
    loss_ref, g_ref = oracle.loss_and_grad(psi_np, tau, dx, 1.0, t, lam)
    assert abs(loss.item() - loss_ref) <= 1e-12 * abs(loss_ref)
    assert rel(g, g_ref) <= 1e-12
    # central finite differences (h = 1e-3) on a few components
    h = 1e-3
    rng = np.random.default_rng(3)
    for _ in range(4):
        i = tuple(int(rng.integers(0, s)) for s in shape)
        for unit, comp in ((1.0, g[i].real), (1j, g[i].imag)):
            vals = []
            for sgn in (+1, -1):
                pp = psi_np.copy()
                pp[i] += sgn * h * unit
                r = fx.expand_density(torch.from_numpy(pp).cuda(), dx, 1.0, t, lam)
                vals.append(((r - tau_t) ** 2).sum().item())
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - comp) <= 1e-6 * max(1.0, abs(comp))


def test_autograd_gradcheck_tiny(fx):
    say("gradcheck")
    psi = torch.from_numpy(workloads.random_field((6, 5), 5)).cuda().requires_grad_(True)

    def f(x):
        return fx.expand_density(x, (1.0, 1.0), 1.0, 2.0, (2, 3))

    assert torch.autograd.gradcheck(f, (psi,), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_column_density_and_density(fx, dtype):
    shape, lam, dx, t = (8, 12, 20), (3, 2, 4), (0.5, 1.0, 1.0), 4.0
    say("column density", dtype)
    psi_np = workloads.random_field(shape, 51)
    psi = torch.from_numpy(psi_np).to(dtype).cuda()
    plan = fx.get_plan(shape, dx, 1.0, t, lam, dtype=dtype)
    out, rho = plan.expand(psi)
    ref_rho = oracle.density(oracle.expand(psi.cpu().numpy().astype(np.complex128), dx, 1.0, t, lam))
    tol = TOL64 if dtype == torch.complex128 else TOL32_RHO
    for axis in range(3):
        img = plan.column_density(rho, axis).cpu().numpy()
        ref_img = oracle.column_density(ref_rho, axis, lam, dx)
        assert rel(img, ref_img) <= tol
    r2 = plan.density(out).cpu().numpy()
    assert rel(r2, rho.cpu().numpy()) <= 1e-15 if dtype == torch.complex128 else 1e-7


def test_torch_owned_workspace(fx):
    shape, lam = (32, 24), (4, 3)
    psi_np = workloads.random_field(shape, 61)
    plan = fx.Plan(shape, (1.0, 1.0), 1.0, 10.0, lam)
    plan.use_torch_workspace()
    out, _ = plan.expand(torch.from_numpy(psi_np).cuda())
    assert rel(out.cpu().numpy(), oracle.expand(psi_np, (1.0, 1.0), 1.0, 10.0, lam)) <= TOL64


def test_small_workspace_budget_forces_blocking(fx, monkeypatch):
    # a tiny budget makes the plan sum the outermost magnification index in several blocks
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    shape, lam = (40, 64, 48), (3, 4, 6)
    say("blocking", shape, lam)
    psi_np = workloads.random_field(shape, 71)
    plan = fx.Plan(shape, (1.0, 1.0, 1.0), 1.0, 8.0, lam)
    import json
    desc = json.loads(plan.describe())
    assert desc["outer_block"] < 6
    out, _ = plan.expand(torch.from_numpy(psi_np).cuda())
    assert rel(out.cpu().numpy(), oracle.expand(psi_np, (1.0,) * 3, 1.0, 8.0, lam)) <= TOL64


def test_batch_ragged_matches_single_plans_and_replays(fx):
    shapes = [(12, 10, 16), (8, 8, 24), (12, 10, 16), (8, 8, 24), (12, 10, 16)]
    lam = (2, 3, 4)
    say("batch", shapes)
    specs = [dict(shape=s, dx=(1.0, 1.0, 1.0), lam=lam, t=9.0) for s in shapes]
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        fields = [workloads.random_field(s, 300 + i) for i, s in enumerate(shapes)]
        psis = [torch.from_numpy(f).to(dtype).cuda() for f in fields]
        b = fx.Batch(specs, dtype=dtype)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            outs, rhos = b.run(psis)
        stream.synchronize()
        for i, (f, s) in enumerate(zip(fields, shapes)):
            ref = oracle.expand(psis[i].cpu().numpy().astype(np.complex128), (1.0,) * 3, 1.0, 9.0, lam)
            if dtype == torch.complex128:
                assert rel(outs[i].cpu().numpy(), ref) <= tol
            assert rel(rhos[i].cpu().numpy(), oracle.density(ref)) <= tol
        first = [o.cpu().numpy().copy() for o in outs]
        # replays of the captured graph, with eager work in between, reproduce the first run
        for rep in range(3):
            with torch.cuda.stream(stream):
                for o in outs:
                    o.zero_()
                _ = fx.expand(psis[0], (1.0,) * 3, 1.0, 9.0, lam)
                b.run(psis, psi_outs=outs, rho_outs=rhos)
            stream.synchronize()
            for i in range(len(shapes)):
                assert np.array_equal(outs[i].cpu().numpy(), first[i])


def test_batch_with_register_passes_matches_oracle(fx):
    # a ragged batch whose classes run the register kernels, the fused structured EA pass
    # (64-point axis, g = 8, P = 8) and the register EA pass (32-point axis, P = 4), in one graph
    shapes = [(64, 6, 8), (32, 6, 8), (64, 6, 8)]
    lam = (8, 2, 2)
    say("batch register passes", shapes)
    specs = [dict(shape=s, dx=(1.0, 1.0, 1.0), lam=lam, t=11.0) for s in shapes]
    fields = [workloads.random_field(s, 700 + i) for i, s in enumerate(shapes)]
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        psis = [torch.from_numpy(f).to(dtype).cuda() for f in fields]
        b = fx.Batch(specs, dtype=dtype)
        outs, rhos = b.run(psis)
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            ref = oracle.expand(psis[i].cpu().numpy().astype(np.complex128), (1.0,) * 3, 1.0, 11.0, lam)
            if dtype == torch.complex128:
                assert rel(outs[i].cpu().numpy(), ref) <= tol
            assert rel(rhos[i].cpu().numpy(), oracle.density(ref)) <= tol


def test_batch_rejects_bad_arguments(fx):
    with pytest.raises(ValueError):
        fx.Batch([dict(shape=(8,), dx=1.0, lam=2, t=1.0), dict(shape=(8,), dx=1.0, lam=0, t=1.0)])
    b = fx.Batch([dict(shape=(8,), dx=1.0, lam=2, t=1.0)], dtype=torch.complex128)
    with pytest.raises(ValueError):
        b.run([torch.zeros(9, dtype=torch.complex128, device="cuda")])


REG_AA_CASES = [
    # shape, lam, dtype: the last two axes with g_u = g_v = 16 or 32 take the register form of
    # the fused accumulate (k_AAR) by default
    ((64, 64), (32, 32), torch.complex128),     # g = 32, P = 2
    ((64, 64), (32, 32), torch.complex64),
    ((128, 128), (16, 16), torch.complex128),   # g = 16, P = 8, four groups per workgroup
    ((128, 128), (16, 16), torch.complex64),
    ((64, 128), (16, 48), torch.complex128),    # P_u = 4, P_v = 8, three terms per residue on v
    ((6, 64, 64), (3, 32, 32), torch.complex128),  # an axis before the fused pair
    ((512, 512), (32, 32), torch.complex64),    # the 512^2, lambda 32 workload
]


@pytest.mark.parametrize("case", range(len(REG_AA_CASES)))
def test_register_two_axis_accumulate_matches_oracle(fx, case, monkeypatch):
    monkeypatch.setenv("FX_NO_EAS", "1")
    shape, lam, dtype = REG_AA_CASES[case]
    dx = (1.0,) * len(shape)
    say("register fused accumulate", shape, lam, dtype)
    psi_np = workloads.random_field(shape, 950 + case)
    if dtype == torch.complex64:
        psi_np = psi_np.astype(np.complex64).astype(np.complex128)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + 0.3
    ref = oracle.expand(psi_np, dx, 1.0, 17.0, lam, a, abar)
    plan = fx.Plan(shape, dx, 1.0, 17.0, lam, list(a), list(abar), dtype)
    import json
    ops = json.loads(plan.describe())["passes"]
    assert ops[-1]["kind"] == "AA" and ops[-1]["g"] == ops[-1]["g2"] == max(np.gcd(lam[-1], shape[-1]), 1)
    out, rho = plan.expand(torch.from_numpy(psi_np).to(dtype).cuda())
    torch.cuda.synchronize()
    if dtype == torch.complex128:
        assert rel(out.cpu().numpy(), ref) <= TOL64
        assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL64
    else:
        assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL32_RHO


def test_register_two_axis_accumulate_blocked(fx, monkeypatch):
    # a tiny workspace splits the outer magnification index into blocks: the fused pass then runs
    # per block with fewer than g terms on v, a first index that is not a multiple of g, accumulating
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    monkeypatch.setenv("FX_NO_EAS", "1")
    shape, lam, dx = (256, 512), (32, 32), (1.0, 1.0)
    say("register fused accumulate blocked", shape, lam)
    psi_np = workloads.random_field(shape, 961)
    ref = oracle.expand(psi_np, dx, 1.0, 13.0, lam)
    plan = fx.Plan(shape, dx, 1.0, 13.0, lam)
    import json
    d = json.loads(plan.describe())
    assert d["outer_block"] < 32
    assert d["passes"][-1]["kind"] == "AA"
    out, rho = plan.expand(torch.from_numpy(psi_np).cuda())
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), ref) <= TOL64
    assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL64


@pytest.mark.parametrize("case", range(len(REG_AA_CASES)))
def test_register_two_axis_adjoint_matches_oracle(fx, case):
    # the adjoint schedule starts with the two AH passes of the same pair, fused (k_AAHR)
    shape, lam, dtype = REG_AA_CASES[case]
    dx = (1.0,) * len(shape)
    say("register fused adjoint accumulate", shape, lam, dtype)
    y_np = workloads.random_field(shape, 970 + case)
    if dtype == torch.complex64:
        y_np = y_np.astype(np.complex64).astype(np.complex128)
    plan = fx.Plan(shape, dx, 1.0, 17.0, lam, dtype=dtype)
    import json
    ops = json.loads(plan.describe())["adjoint_passes"]
    assert ops[0]["kind"] == "AAH"
    g = plan.expand_adjoint(torch.from_numpy(y_np).to(dtype).cuda()).cpu().numpy()
    ref = oracle.expand_adjoint(y_np, dx, 1.0, 17.0, lam)
    assert rel(g, ref) <= (TOL64 if dtype == torch.complex128 else TOL32_RHO)


def test_register_two_axis_adjoint_blocked(fx, monkeypatch):
    # blocks of the outer magnification index: the fused adjoint pass runs per block with fewer
    # than g terms on v and a first index that is not a multiple of g
    monkeypatch.setenv("FX_WORKSPACE_MB", "1")
    shape, lam, dx = (256, 512), (32, 32), (1.0, 1.0)
    say("register fused adjoint blocked", shape, lam)
    y_np = workloads.random_field(shape, 980)
    plan = fx.Plan(shape, dx, 1.0, 13.0, lam)
    import json
    d = json.loads(plan.describe())
    assert d["outer_block"] < 32 and d["adjoint_passes"][0]["kind"] == "AAH"
    g = plan.expand_adjoint(torch.from_numpy(y_np).cuda()).cpu().numpy()
    assert rel(g, oracle.expand_adjoint(y_np, dx, 1.0, 13.0, lam)) <= TOL64


def test_register_two_axis_accumulate_term_ranges(fx, monkeypatch):
    # ranges of the flat term index decompose into blocks whose first indices on both axes are not
    # multiples of g = 32 and that hold 1..32 terms per axis
    monkeypatch.setenv("FX_NO_EAS", "1")
    shape, lam, dx, t = (64, 64), (32, 32), (1.0, 1.0), 9.0
    say("register fused accumulate ranges", shape, lam)
    psi_np = workloads.random_field(shape, 962)
    psi = torch.from_numpy(psi_np).cuda()
    plan = fx.Plan(shape, dx, 1.0, t, lam)
    acc = torch.zeros_like(psi)
    cuts = [0, 5, 37, 100, 640, 1000, 1024]
    for b, e in zip(cuts[:-1], cuts[1:]):
        plan.expand_range(psi, acc, b, e, accumulate=True)
    torch.cuda.synchronize()
    assert rel(acc.cpu().numpy(), oracle.expand(psi_np, dx, 1.0, t, lam)) <= TOL64


@pytest.mark.parametrize("case", [5, 7, 9, 15, 19, 22])
def test_fused_two_axis_accumulate_fp64(fx, case, monkeypatch):
    # the optional fused form of the last two accumulate passes (FX_AA=1), read at plan creation;
    # the structured EA pass, which leaves a single accumulate pass, is switched off for it
    monkeypatch.setenv("FX_AA", "1")
    monkeypatch.setenv("FX_NO_EAS", "1")
    shape, lam, dx, t, moh, shift = CASES[case]
    say("fused accumulate", shape, lam)
    psi_np = workloads.random_field(shape, 900 + case)
    a, abar = oracle.default_offsets(shape, dx, lam)
    abar = abar + shift * np.asarray(dx)
    ref = oracle.expand(psi_np, dx, moh, t, lam, a, abar)
    plan = fx.Plan(shape, dx, moh, t, lam, list(a), list(abar), torch.complex128)
    assert '"AA"' in plan.describe() or len(shape) == 1
    out, rho = plan.expand(torch.from_numpy(psi_np).cuda())
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), ref) <= TOL64
    assert rel(rho.cpu().numpy(), oracle.density(ref)) <= TOL64
