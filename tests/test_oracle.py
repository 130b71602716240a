"""Pins for the CPU oracle: closed forms, invariants, finite differences and
independent library routines.  None of these re-types the oracle's own
formulas; each would fail for a plausible mistake in it (dropped term, wrong
sign or index, transposed operand, wrong mask)."""

import dataclasses

import numpy as np
import pytest

import oracle
import synth
from synth.grids import Grid

PQ, PV, SLACK = 0, 1, 2


def two_bus(r, x, v1, P, Q):
    """Slack (bus 0, |V|=v1, angle 0) -- one branch r+jx (no charging) -- PQ bus 1."""
    return Grid(2, np.array([0], np.int32), np.array([1], np.int32), np.array([r]),
                np.array([x]), np.array([0.0]), np.array([SLACK, PQ], np.int8),
                np.array([v1, 1.0]), np.array([0.0, 0.0]))


def two_bus_closed_form(r, x, v1, P, Q):
    """High-voltage root of the 2-bus power flow.

    With c = conj(z) S2 and W = |V2|^2, the PQ bus satisfies
    W - v1 V2 = c, hence (W - c_r)^2 + c_i^2 = W v1^2, a quadratic in W."""
    c = np.conj(r + 1j * x) * (P + 1j * Q)
    bq = 2 * c.real + v1 ** 2
    W = (bq + np.sqrt(bq ** 2 - 4 * (c.real ** 2 + c.imag ** 2))) / 2
    return (W - c) / v1


CASES_2BUS = [(0.05, 0.2, 1.02, -0.8, -0.3), (0.02, 0.1, 1.0, -1.5, -0.2),
              (0.1, 0.3, 0.98, 0.4, 0.1), (0.01, 0.05, 1.05, -2.0, 0.5)]


@pytest.mark.parametrize("r,x,v1,P,Q", CASES_2BUS)
def test_two_bus_closed_form_mismatch(r, x, v1, P, Q):
    g = two_bus(r, x, v1, P, Q)
    Y = oracle.ybus_of(g)
    V2 = two_bus_closed_form(r, x, v1, P, Q)
    vm = np.array([v1, abs(V2)])
    va = np.array([0.0, np.angle(V2)])
    S = np.array([0.0, P + 1j * Q])
    dS = oracle.mismatch(Y, vm, va, S)
    assert abs(dS[1]) < 1e-13
    loss, mu, gvm, gva = oracle.loss_grad(Y, g.bus_type, vm, va, S)
    assert mu < 1e-13 and loss < 1e-26
    assert np.abs(gvm).max() < 1e-12 and np.abs(gva).max() < 1e-12


@pytest.mark.parametrize("r,x,v1,P,Q", CASES_2BUS)
def test_two_bus_newton_and_adam_reach_closed_form(r, x, v1, P, Q):
    g = two_bus(r, x, v1, P, Q)
    Y = oracle.ybus_of(g)
    V2 = two_bus_closed_form(r, x, v1, P, Q)
    S = np.array([0.0, P + 1j * Q])
    nr = oracle.newton(Y, g.bus_type, S, np.array([v1, 1.0]), np.zeros(2), tol=1e-12)
    assert nr["converged"]
    assert abs(nr["vm"][1] * np.exp(1j * nr["va"][1]) - V2) < 1e-10
    res = oracle.solve_adam(Y, g.bus_type, S, np.array([v1, 1.0]), np.zeros(2),
                            oracle.AdamOptions(lr=1e-3, tol=1e-9, max_iter=200000))
    assert res["status"] == 0
    assert abs(res["vm"][1] * np.exp(1j * res["va"][1]) - V2) < 1e-8


def branch_flow_injections(g, vm, va):
    """Nodal injections as the sum of pi-model branch end flows (independent of Y)."""
    V = vm * np.exp(1j * va)
    S = np.zeros(g.n_bus, dtype=complex)
    for e in range(g.n_branch):
        f, t = g.f[e], g.t[e]
        y = 1 / (g.r[e] + 1j * g.x[e])
        i_f = y * (V[f] - V[t]) + 0.5j * g.b[e] * V[f]
        i_t = y * (V[t] - V[f]) + 0.5j * g.b[e] * V[t]
        S[f] += V[f] * np.conj(i_f)
        S[t] += V[t] * np.conj(i_t)
    return S


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_zero_against_branch_flows(seed):
    g = synth.config0(seed)["grid"]
    Y = oracle.ybus_of(g)
    S = branch_flow_injections(g, g.vm, g.va)
    dS = oracle.mismatch(Y, g.vm, g.va, S)
    assert np.abs(dS).max() < 1e-13
    loss, mu, gvm, gva = oracle.loss_grad(Y, g.bus_type, g.vm, g.va, S)
    assert mu < 1e-13
    assert max(np.abs(gvm).max(), np.abs(gva).max()) < 1e-12


def test_planted_zero_meshed_grid():
    g = synth.config1(B=1)["grid"]
    Y = oracle.ybus_of(g)
    S = branch_flow_injections(g, g.vm, g.va)
    dS = oracle.mismatch(Y, g.vm, g.va, S)
    assert np.abs(dS).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 3])
def test_power_balance(seed):
    """Sum of injections = sum of branch losses r|I|^2 + j(x|I|^2 - b/2(|Vf|^2+|Vt|^2))."""
    g = synth.config0(seed)["grid"]
    Y = oracle.ybus_of(g)
    rng = np.random.default_rng(seed)
    vm = g.vm + rng.normal(0, 0.03, g.n_bus)
    va = g.va + rng.normal(0, 0.05, g.n_bus)
    S = oracle.injections(Y, vm, va)
    V = vm * np.exp(1j * va)
    Is = (V[g.f] - V[g.t]) / (g.r + 1j * g.x)
    loss_p = np.sum(g.r * np.abs(Is) ** 2)
    loss_q = np.sum(g.x * np.abs(Is) ** 2 - 0.5 * g.b * (np.abs(V[g.f]) ** 2 + np.abs(V[g.t]) ** 2))
    assert abs(S.sum().real - loss_p) < 1e-12 * max(1, loss_p)
    assert abs(S.sum().imag - loss_q) < 1e-12 * max(1, abs(loss_q))
    assert S.sum().real >= 0


def test_ybus_invariants():
    g = synth.config1(B=1)["grid"]
    Y = oracle.ybus_of(g)
    # rows sorted, diagonal present, no duplicate columns
    for i in range(g.n_bus):
        cols = Y.col[Y.row_ptr[i]:Y.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    import scipy.sparse as sp
    A = sp.csr_matrix((Y.val, Y.col, Y.row_ptr), shape=(g.n_bus, g.n_bus))
    assert abs(A - A.T).max() == 0.0  # complex symmetric
    rowsum = A @ np.ones(g.n_bus)
    half_b = np.zeros(g.n_bus)
    np.add.at(half_b, g.f, g.b / 2)
    np.add.at(half_b, g.t, g.b / 2)
    assert np.abs(rowsum - 1j * half_b).max() < 1e-12
    assert Y.nnz == g.n_bus + 2 * g.n_branch  # no parallel branches in the generator


def test_ybus_parallel_branches_and_skip():
    g = synth.config0(4)["grid"]
    # duplicate branch 3: two parallel branches must sum into the same entries
    f = np.append(g.f, g.f[3]); t = np.append(g.t, g.t[3])
    r = np.append(g.r, 0.07); x = np.append(g.x, 0.11); b = np.append(g.b, 0.02)
    Y2 = oracle.build_ybus(g.n_bus, f, t, r, x, b)
    assert Y2.nnz == oracle.ybus_of(g).nnz
    # skipping the appended branch equals the original grid exactly
    Ys = oracle.build_ybus(g.n_bus, f, t, r, x, b, skip=len(f) - 1)
    Y0 = oracle.ybus_of(g)
    assert np.array_equal(Ys.col, Y0.col) and np.allclose(Ys.val, Y0.val, rtol=0, atol=1e-15)
    # skip = deleting the branch from the input arrays
    k = 5
    keep = np.arange(g.n_branch) != k
    Yd = oracle.build_ybus(g.n_bus, g.f[keep], g.t[keep], g.r[keep], g.x[keep], g.b[keep])
    Yk = oracle.ybus_of(g, skip=k)
    assert np.allclose(Yd.dense(), Yk.dense(), rtol=0, atol=1e-15)


def test_ybus_rejects_bad_input():
    with pytest.raises(oracle.OracleError):
        oracle.build_ybus(3, [0], [0], [0.1], [0.1], [0.0])  # self loop
    with pytest.raises(oracle.OracleError):
        oracle.build_ybus(3, [0], [3], [0.1], [0.1], [0.0])  # out of range
    with pytest.raises(oracle.OracleError):
        oracle.build_ybus(3, [0], [1], [0.0], [0.0], [0.0])  # zero impedance


def _fd_grad(Y, bt, vm, va, S, h=1e-6, coords=None):
    n = len(vm)
    coords = range(n) if coords is None else coords
    gv, ga = {}, {}
    for i in coords:
        e = np.zeros(n); e[i] = h
        gv[i] = (oracle.loss_grad(Y, bt, vm + e, va, S)[0] - oracle.loss_grad(Y, bt, vm - e, va, S)[0]) / (2 * h)
        ga[i] = (oracle.loss_grad(Y, bt, vm, va + e, S)[0] - oracle.loss_grad(Y, bt, vm, va - e, S)[0]) / (2 * h)
    return gv, ga


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_gradient_matches_central_fd_all_coordinates(seed):
    g = synth.config0(seed)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    rng = np.random.default_rng(100 + seed)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    _, _, gvm, gva = oracle.loss_grad(Y, g.bus_type, vm, va, S)
    fv, fa = _fd_grad(Y, g.bus_type, vm, va, S)
    scale = max(np.abs(gvm).max(), np.abs(gva).max())
    for i in range(g.n_bus):
        ev = fv[i] if g.bus_type[i] == PQ else 0.0
        ea = fa[i] if g.bus_type[i] != SLACK else 0.0
        assert abs(gvm[i] - ev) <= 1e-6 * scale
        assert abs(gva[i] - ea) <= 1e-6 * scale


def test_gradient_matches_fd_meshed_sampled():
    cfg = synth.config1(B=2)
    g = cfg["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va) * cfg["load_scale"][1]
    rng = np.random.default_rng(7)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    _, _, gvm, gva = oracle.loss_grad(Y, g.bus_type, vm, va, S)
    learn_v = np.flatnonzero(g.bus_type == PQ)
    learn_a = np.flatnonzero(g.bus_type != SLACK)
    cv = rng.choice(learn_v, 32, replace=False)
    ca = rng.choice(learn_a, 32, replace=False)
    fv, _ = _fd_grad(Y, g.bus_type, vm, va, S, coords=cv)
    _, fa = _fd_grad(Y, g.bus_type, vm, va, S, coords=ca)
    for i in cv:
        assert abs(gvm[i] - fv[i]) <= 1e-6 * max(abs(fv[i]), 1e-3 * np.abs(gvm).max())
    for i in ca:
        assert abs(gva[i] - fa[i]) <= 1e-6 * max(abs(fa[i]), 1e-3 * np.abs(gva).max())


def test_nr_jacobian_matches_fd():
    g = synth.config0(2)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    rng = np.random.default_rng(3)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    J, pvpq, pq = oracle.jacobian_f(Y, g.bus_type, vm, va)
    J = J.toarray()
    h = 1e-6
    cols = [("a", i) for i in pvpq] + [("m", i) for i in pq]
    for k, (kind, i) in enumerate(cols):
        e = np.zeros(g.n_bus); e[i] = h
        if kind == "a":
            fp = oracle.residual_vector(Y, g.bus_type, vm, va + e, S)
            fm = oracle.residual_vector(Y, g.bus_type, vm, va - e, S)
        else:
            fp = oracle.residual_vector(Y, g.bus_type, vm + e, va, S)
            fm = oracle.residual_vector(Y, g.bus_type, vm - e, va, S)
        assert np.abs((fp - fm) / (2 * h) - J[:, k]).max() < 1e-7 * np.abs(J).max()


def test_newton_quadratic_convergence_to_planted():
    cfg = synth.config1(B=1)
    g = cfg["grid"]
    Y = oracle.ybus_of(g)
    S = branch_flow_injections(g, g.vm, g.va)
    rng = np.random.default_rng(11)
    vm0 = g.vm.copy(); va0 = g.va.copy()
    vm0[g.bus_type == PQ] += rng.normal(0, 1e-3, int((g.bus_type == PQ).sum()))
    va0[g.bus_type != SLACK] += rng.normal(0, 1e-3, g.n_bus - 1)
    nr = oracle.newton(Y, g.bus_type, S, vm0, va0, tol=1e-11)
    assert nr["converged"] and nr["iters"] <= 5
    h = nr["history"]
    # quadratic: once in the basin, each error is bounded by C * previous^2
    # (a wrong Jacobian entry degrades this to linear convergence, for which
    # the ratio grows like 1/e_k)
    checked = 0
    for k in range(1, len(h) - 1):
        if h[k] < 1e-3 and h[k + 1] > 1e-13:
            assert h[k + 1] <= 1e3 * h[k] ** 2
            checked += 1
    assert checked >= 1
    assert np.abs(nr["vm"] - g.vm).max() < 1e-9
    assert np.abs(nr["va"] - g.va).max() < 1e-9


def test_newton_flat_start_finds_planted_small():
    cfg = synth.config0(0)
    g = cfg["grid"]
    Y = oracle.ybus_of(g)
    S = branch_flow_injections(g, g.vm, g.va)
    nr = oracle.newton(Y, g.bus_type, S, cfg["vm0"][0], cfg["va0"][0], tol=1e-10)
    assert nr["converged"]
    assert np.abs(nr["vm"] - g.vm).max() < 1e-8


def test_gradient_equals_scaled_jt_f():
    """Sec. 5.1: dL/dx = (2/m) J_f^T f, with J_f assembled from Algorithm 2."""
    cfg = synth.config1(B=1)
    g = cfg["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    rng = np.random.default_rng(5)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    J, pvpq, pq = oracle.jacobian_f(Y, g.bus_type, vm, va)
    f = oracle.residual_vector(Y, g.bus_type, vm, va, S)
    m = len(f)
    assert m == oracle.residual_count(g.bus_type) == len(pvpq) + len(pq)
    gx = (2.0 / m) * (J.T @ f)
    _, _, gvm, gva = oracle.loss_grad(Y, g.bus_type, vm, va, S)
    scale = np.abs(gx).max()
    assert np.abs(gva[pvpq] - gx[:len(pvpq)]).max() < 1e-12 * scale
    assert np.abs(gvm[pq] - gx[len(pvpq):]).max() < 1e-12 * scale
    assert np.all(gvm[g.bus_type != PQ] == 0) and np.all(gva[g.bus_type == SLACK] == 0)
    loss, mu = oracle.loss_from_mismatch(g.bus_type, oracle.mismatch(Y, vm, va, S))
    assert abs(loss - np.mean(f ** 2)) < 1e-14 * loss
    assert mu == np.abs(f).max()


def _torch_adam_reference(Y, bt, S, vm0, va0, steps, lr, betas, eps, plateau=None, step_lr=None):
    """Same iteration driven by torch.optim.Adam (and optionally torch's
    ReduceLROnPlateau or StepLR) with gradients from the oracle."""
    torch = pytest.importorskip("torch")
    vm = torch.tensor(vm0, dtype=torch.float64)
    va = torch.tensor(va0, dtype=torch.float64)
    pv = torch.nn.Parameter(vm.clone())
    pa = torch.nn.Parameter(va.clone())
    opt = torch.optim.Adam([pv, pa], lr=lr, betas=betas, eps=eps)
    sch = None
    if plateau is not None:
        sch = torch.optim.lr_scheduler.ReduceLROnPlateau(opt, mode="min", **plateau)
    if step_lr is not None:
        sch = torch.optim.lr_scheduler.StepLR(opt, **step_lr)
    lrs = []
    for _ in range(steps):
        loss, mu, gvm, gva = oracle.loss_grad(Y, bt, pv.detach().numpy(), pa.detach().numpy(), S)
        pv.grad = torch.tensor(gvm)
        pa.grad = torch.tensor(gva)
        opt.step()
        if plateau is not None:
            sch.step(loss)
        elif sch is not None:
            sch.step()
        lrs.append(opt.param_groups[0]["lr"])
    return pv.detach().numpy(), pa.detach().numpy(), lrs


def _torch_opt_reference(Y, bt, S, vm0, va0, steps, make_opt):
    """The same iteration driven by a torch.optim optimizer on the oracle's gradients."""
    torch = pytest.importorskip("torch")
    pv = torch.nn.Parameter(torch.tensor(vm0, dtype=torch.float64))
    pa = torch.nn.Parameter(torch.tensor(va0, dtype=torch.float64))
    opt = make_opt([pv, pa])
    for _ in range(steps):
        _, _, gvm, gva = oracle.loss_grad(Y, bt, pv.detach().numpy(), pa.detach().numpy(), S)
        pv.grad = torch.tensor(gvm)
        pa.grad = torch.tensor(gva)
        opt.step()
    return pv.detach().numpy(), pa.detach().numpy()


@pytest.mark.parametrize("kind", ["sgd", "sgd_momentum", "rmsprop"])
def test_sgd_and_rmsprop_match_torch_optim(kind):
    """The paper's other optimizers (Sec. 6.3: SGD and RMSprop) with PyTorch's
    definitions: SGD with momentum beta1 (buffer = first gradient, no
    dampening), RMSprop with smoothing beta2 and eps outside the root."""
    torch = pytest.importorskip("torch")
    g = synth.config0(1)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    # short enough that no coordinate has started to oscillate about its
    # solution (there the sign-like steps amplify rounding differences)
    steps = 50 if kind == "rmsprop" else 200
    if kind == "rmsprop":
        o = oracle.AdamOptions(lr=1e-3, beta2=0.99, eps=1e-8, tol=0.0, max_iter=steps,
                               optimizer=oracle.OPT_RMSPROP)
        make = lambda p: torch.optim.RMSprop(p, lr=1e-3, alpha=0.99, eps=1e-8)
    else:
        mom = 0.9 if kind == "sgd_momentum" else 0.0
        o = oracle.AdamOptions(lr=3e-3, beta1=mom, tol=0.0, max_iter=steps, optimizer=oracle.OPT_SGD)
        make = lambda p: torch.optim.SGD(p, lr=3e-3, momentum=mom)
    ref_vm, ref_va = _torch_opt_reference(Y, g.bus_type, S, vm0, va0, steps, make)
    res = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o)
    assert res["iters"] == steps
    assert np.abs(res["vm"] - ref_vm).max() < 1e-12
    assert np.abs(res["va"] - ref_va).max() < 1e-12
    # the iteration moved: the pin is not satisfied by a no-op update
    assert np.abs(res["va"] - va0).max() > 1e-3


def test_adam_matches_torch_optim():
    g = synth.config0(1)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    steps = 300
    ref_vm, ref_va, _ = _torch_adam_reference(Y, g.bus_type, S, vm0, va0, steps, 1e-2, (0.9, 0.999), 1e-8)
    res = oracle.solve_adam(Y, g.bus_type, S, vm0, va0,
                            oracle.AdamOptions(lr=1e-2, tol=0.0, max_iter=steps))
    assert res["status"] == 1 and res["iters"] == steps
    assert np.abs(res["vm"] - ref_vm).max() < 1e-11
    assert np.abs(res["va"] - ref_va).max() < 1e-11
    # fixed coordinates never move
    assert np.all(res["vm"][g.bus_type != PQ] == vm0[g.bus_type != PQ])
    assert res["va"][g.bus_type == SLACK][0] == 0.0


def test_plateau_schedule_matches_torch():
    g = synth.config0(2)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    steps = 600
    pl = dict(factor=0.547, patience=41, threshold=0.0673, cooldown=97)
    ref_vm, ref_va, lrs = _torch_adam_reference(Y, g.bus_type, S, vm0, va0, steps, 1e-2,
                                                (0.979, 0.963), 1e-8, plateau=pl)
    assert min(lrs) < 1e-2  # the schedule did act
    o = oracle.AdamOptions(lr=1e-2, beta1=0.979, beta2=0.963, tol=0.0, max_iter=steps,
                           sched=oracle.SCHED_PLATEAU, **pl)
    res = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o)
    assert abs(res["lr"] - lrs[-1]) <= 1e-15
    assert np.abs(res["vm"] - ref_vm).max() < 1e-9
    assert np.abs(res["va"] - ref_va).max() < 1e-9


@pytest.mark.parametrize("min_lr,sched_eps", [(3e-3, 1e-8), (0.0, 3e-3)])
def test_plateau_clamp_and_eps_guard_match_torch(min_lr, sched_eps):
    """ReduceLROnPlateau's lower bound (min_lr) and its skip of small decreases
    (eps) at values where each of them acts: with min_lr = 3e-3 the second
    decrease is clamped to it and later ones are no-ops; with eps = 3e-3 the
    first decrease (1e-2 -> 5.47e-3) applies and the second (by 2.5e-3) is
    skipped."""
    g = synth.config0(2)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    # 500 steps: plateaus end at steps 55, 211 and 418 with the default bounds
    steps = 500
    pl = dict(factor=0.547, patience=41, threshold=0.0673, cooldown=97)
    ref_vm, ref_va, lrs = _torch_adam_reference(Y, g.bus_type, S, vm0, va0, steps, 1e-2, (0.979, 0.963), 1e-8,
                                                plateau=dict(pl, min_lr=min_lr, eps=sched_eps))
    if min_lr > 0:
        assert lrs[-1] == min_lr and 1e-2 * 0.547 in lrs  # clamped after a plain decrease
    else:
        assert lrs[-1] == 1e-2 * 0.547  # the second decrease was skipped
    o = oracle.AdamOptions(lr=1e-2, beta1=0.979, beta2=0.963, tol=0.0, max_iter=steps,
                           sched=oracle.SCHED_PLATEAU, min_lr=min_lr, sched_eps=sched_eps, **pl)
    res = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o)
    assert res["lr"] == lrs[-1]
    assert np.abs(res["vm"] - ref_vm).max() < 1e-11
    assert np.abs(res["va"] - ref_va).max() < 1e-11


def test_step_schedule_matches_torch_and_resumes():
    """StepLR (Table 3's first time step; one of the schedulers searched in
    Sec. 6.3) against torch.optim.lr_scheduler.StepLR on the oracle's gradients,
    run in one call and as two resumed calls whose split (37) is not a multiple of
    the step size (30): the decay follows the persistent step count, so the
    second call keeps the phase."""
    g = synth.config0(1)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    steps, size, gamma = 100, 30, 0.773
    ref_vm, ref_va, lrs = _torch_adam_reference(Y, g.bus_type, S, vm0, va0, steps, 1e-2, (0.9802, 0.944), 1e-8,
                                                step_lr=dict(step_size=size, gamma=gamma))
    assert lrs[-1] == pytest.approx(1e-2 * gamma ** 3, rel=1e-15)
    o = oracle.AdamOptions(lr=1e-2, beta1=0.9802, beta2=0.944, tol=0.0, max_iter=steps,
                           sched=oracle.SCHED_STEP, factor=gamma, patience=size)
    res = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o)
    assert res["iters"] == steps and res["t"] == steps
    assert res["lr"] == lrs[-1]
    assert np.abs(res["vm"] - ref_vm).max() < 1e-11
    assert np.abs(res["va"] - ref_va).max() < 1e-11
    # two resumed calls: moments, step count and current lr carried over
    k1 = 37
    r1 = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, dataclasses.replace(o, max_iter=k1))
    assert r1["lr"] == lrs[k1 - 1] and r1["t"] == k1
    r2 = oracle.solve_adam(Y, g.bus_type, S, r1["vm"], r1["va"],
                           dataclasses.replace(o, lr=r1["lr"], max_iter=steps - k1), state=r1["state"], t0=r1["t"])
    assert r2["t"] == steps and r2["lr"] == res["lr"]
    assert np.array_equal(r2["vm"], res["vm"]) and np.array_equal(r2["va"], res["va"])
    # a call that restarted the phase at the split would decay at 37 + 30 = 67, not at 60
    assert lrs[59] < lrs[58]


def test_native_build_computes_the_same_iterates():
    """The benchmark's CPU-baseline leg runs the oracle built with -O3
    -march=native for its host; with FP contraction still off it must take the
    pinned build's iterates bit for bit (the baseline times the oracle, not a
    different program)."""
    g = synth.config0(1)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    o = oracle.AdamOptions(lr=1e-2, tol=0.0, max_iter=300, sched=oracle.SCHED_PLATEAU, factor=0.5, patience=20)
    a = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o)
    b = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, o, native=True)
    assert np.array_equal(a["vm"], b["vm"]) and np.array_equal(a["va"], b["va"]) and a["lr"] == b["lr"]


def test_stop_test_semantics():
    g = synth.config0(0)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    r = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, oracle.AdamOptions(tol=1e9, max_iter=10))
    assert r["status"] == 0 and r["iters"] == 0 and np.array_equal(r["vm"], vm0)
    r = oracle.solve_adam(Y, g.bus_type, S, vm0, va0, oracle.AdamOptions(max_iter=0))
    assert r["status"] == 1 and r["iters"] == 0
    Sbad = S.copy(); Sbad[3] = np.nan
    r = oracle.solve_adam(Y, g.bus_type, Sbad, vm0, va0, oracle.AdamOptions(max_iter=10))
    assert r["status"] == 2 and r["iters"] == 0
    # converged at the planted point immediately
    r = oracle.solve_adam(Y, g.bus_type, S, g.vm, g.va, oracle.AdamOptions(max_iter=10))
    assert r["status"] == 0 and r["iters"] == 0


def test_batch_equals_single_solves():
    g = synth.config0(0)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    scale = np.random.default_rng(0).uniform(0.95, 1.05, (3, g.n_bus))
    Sb = S[None, :] * scale
    vm0, va0 = synth.flat_start(g)
    o = oracle.AdamOptions(max_iter=500)
    vb = np.tile(vm0, (3, 1)); ab = np.tile(va0, (3, 1))
    res = oracle.solve_adam_batch(Y, g.bus_type, Sb, vb, ab, o)
    for c in range(3):
        one = oracle.solve_adam(Y, g.bus_type, Sb[c], vm0, va0, o)
        assert np.array_equal(one["vm"], res["vm"][c]) and one["iters"] == res["iters"][c]


def _loss_of(g, bt, vm, va, S, skip=-1):
    Y = oracle.ybus_of(g, skip=skip)
    return oracle.loss_from_mismatch(bt, oracle.mismatch(Y, vm, va, S))[0]


@pytest.mark.parametrize("skip", [-1, 6])
def test_param_grad_matches_central_differences(skip):
    """dL/d(r, x, b) of every branch and dL/dS_spec by central differences of
    the loss (Y rebuilt from the perturbed branch data), with and without an
    outaged branch."""
    import dataclasses
    g = synth.config0(4)["grid"]
    Y = oracle.ybus_of(g, skip=skip)
    S = oracle.injections(oracle.ybus_of(g), g.vm, g.va)
    rng = np.random.default_rng(11)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    g_r, g_x, g_b, g_s = oracle.param_grad(g, g.bus_type, vm, va, S, skip=skip)
    h = 1e-6
    scale = max(np.abs(g_r).max(), np.abs(g_x).max(), np.abs(g_b).max())
    for name, grad in (("r", g_r), ("x", g_x), ("b", g_b)):
        for e in range(g.n_branch):
            arr = getattr(g, name)
            up, dn = arr.copy(), arr.copy()
            up[e] += h
            dn[e] -= h
            fd = (_loss_of(dataclasses.replace(g, **{name: up}), g.bus_type, vm, va, S, skip)
                  - _loss_of(dataclasses.replace(g, **{name: dn}), g.bus_type, vm, va, S, skip)) / (2 * h)
            assert abs(grad[e] - fd) <= 1e-6 * scale, (name, e)
    if skip >= 0:
        assert g_r[skip] == 0.0 and g_x[skip] == 0.0 and g_b[skip] == 0.0
    for i in range(g.n_bus):
        for part in (1.0, 1.0j):
            Su, Sd = S.copy(), S.copy()
            Su[i] += part * h
            Sd[i] -= part * h
            fd = (_loss_of(g, g.bus_type, vm, va, Su, skip) - _loss_of(g, g.bus_type, vm, va, Sd, skip)) / (2 * h)
            an = g_s[i].real if part == 1.0 else g_s[i].imag
            assert abs(an - fd) <= 1e-6 * np.abs(g_s).max()
    # closed form of the injection gradient: -(2/m) times the masked residual
    dS = oracle.mismatch(Y, vm, va, S)
    m = oracle.residual_count(g.bus_type)
    rP = np.where(g.bus_type != SLACK, dS.real, 0.0)
    rQ = np.where(g.bus_type == PQ, dS.imag, 0.0)
    assert np.allclose(g_s, -(2.0 / m) * (rP + 1j * rQ), rtol=0, atol=1e-15)


def test_param_grad_vanishes_at_the_planted_solution():
    g = synth.config1(B=1)["grid"]
    S = oracle.injections(oracle.ybus_of(g), g.vm, g.va)
    g_r, g_x, g_b, g_s = oracle.param_grad(g, g.bus_type, g.vm, g.va, S)
    assert max(np.abs(g_r).max(), np.abs(g_x).max(), np.abs(g_b).max(), np.abs(g_s).max()) < 1e-12


def test_dc_power_flow_two_bus_closed_form():
    """Slack at bus 0, one branch of reactance x: theta_1 = P_1 x."""
    g = synth.Grid(n_bus=2, f=np.array([0], np.int32), t=np.array([1], np.int32), r=np.array([0.02]),
                   x=np.array([0.25]), b=np.array([0.0]), bus_type=np.array([2, 0], np.int8),
                   vm=np.ones(2), va=np.zeros(2))
    th = oracle.dc_power_flow(g, g.bus_type, np.array([0.0, -0.4 + 0.1j]), va_slack=0.1)
    assert th[0] == 0.1 and abs(th[1] - (0.1 - 0.4 * 0.25)) < 1e-15


def test_dc_power_flow_tree_flows_balance_subtree_injections():
    """On a tree the DC branch flow (theta_f - theta_t)/x equals the injection
    total of the subtree behind the branch (flow conservation, no solve)."""
    g = synth.config0(7)["grid"]
    rng = np.random.default_rng(4)
    tree = synth.Grid(n_bus=g.n_bus, f=np.array([rng.integers(0, k) for k in range(1, g.n_bus)], np.int32),
                      t=np.arange(1, g.n_bus, dtype=np.int32), r=np.full(g.n_bus - 1, 0.01),
                      x=rng.uniform(0.05, 0.3, g.n_bus - 1), b=np.zeros(g.n_bus - 1),
                      bus_type=np.where(np.arange(g.n_bus) == 0, 2, 0).astype(np.int8), vm=g.vm, va=g.va)
    P = rng.normal(0, 0.3, g.n_bus)
    th = oracle.dc_power_flow(tree, tree.bus_type, P + 0j)
    children = {k: [] for k in range(g.n_bus)}
    for f, t in zip(tree.f, tree.t):
        children[int(f)].append(int(t))
    def subtree(k):
        return P[k] + sum(subtree(c) for c in children[k])
    for e, (f, t) in enumerate(zip(tree.f, tree.t)):
        flow_into_t = (th[f] - th[t]) / tree.x[e]  # from parent f towards child t
        assert abs(flow_into_t + subtree(int(t))) < 1e-12


def test_dc_power_flow_is_the_small_angle_limit_of_ac():
    """Lossless branches, no charging, all non-slack buses PV at |V| = 1 and
    tiny injections: Newton-Raphson's AC angles approach the DC angles with a
    relative error of second order in the angles."""
    g0 = synth.config0(3)["grid"]
    g = synth.Grid(n_bus=g0.n_bus, f=g0.f, t=g0.t, r=np.zeros(g0.n_branch), x=g0.x, b=np.zeros(g0.n_branch),
                   bus_type=np.where(g0.bus_type == 2, 2, 1).astype(np.int8), vm=np.ones(g0.n_bus),
                   va=np.zeros(g0.n_bus))
    rng = np.random.default_rng(9)
    P = rng.normal(0, 1.0, g.n_bus)
    P[g.bus_type == 2] = 0.0
    P -= P.mean() * (g.bus_type != 2)
    for eps in (1e-2, 1e-3):
        th = oracle.dc_power_flow(g, g.bus_type, eps * P + 0j)
        nr = oracle.newton(oracle.ybus_of(g), g.bus_type, eps * P + 0j, np.ones(g.n_bus), np.zeros(g.n_bus),
                           tol=1e-14)
        assert nr["converged"]
        err = np.abs(nr["va"] - th).max() / np.abs(th).max()
        assert err < 5 * eps ** 2
