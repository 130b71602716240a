"""The plain-autograd comparison system computes the same iterates as the
oracle (CPU torch sparse tensors; no GPU needed)."""

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


def _run(g, S, vm0, va0, opts_kw, outage=None, steps=40):
    from paper_2603_28203_amd.autograd_baseline import AutogradDPF
    from paper_2603_28203_amd.binding import Options

    Y = oracle.ybus_of(g)
    ag = AutogradDPF(Y.row_ptr, Y.col, Y.val, g.n_bus, g.bus_type, S, outage=outage,
                     branch=(g.f, g.t, g.r, g.x, g.b), device="cpu")
    o = Options(**{**opts_kw, "tol": 0.0, "max_iter": steps})
    return ag.solve(torch.tensor(vm0), torch.tensor(va0), o)


def test_autograd_loss_and_gradient_match_oracle():
    from paper_2603_28203_amd.autograd_baseline import AutogradDPF

    g = synth.config0(1)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    rng = np.random.default_rng(0)
    vm = g.vm + rng.normal(0, 0.02, g.n_bus)
    va = g.va + rng.normal(0, 0.02, g.n_bus)
    ag = AutogradDPF(Y.row_ptr, Y.col, Y.val, g.n_bus, g.bus_type, S, device="cpu")
    v = torch.tensor(vm[None], requires_grad=True)
    a = torch.tensor(va[None], requires_grad=True)
    loss, mu = ag.loss(v, a)
    loss.sum().backward()
    lo, muo, gv, ga = oracle.loss_grad(Y, g.bus_type, vm, va, S)
    assert abs(loss.item() - lo) <= 1e-12 * lo and abs(mu.item() - muo) <= 1e-12 * muo
    gvm = v.grad[0].numpy() * (g.bus_type == 0)
    gva = a.grad[0].numpy() * (g.bus_type != 2)
    assert np.abs(gvm - gv).max() <= 1e-10 * np.abs(gv).max()
    assert np.abs(gva - ga).max() <= 1e-10 * np.abs(ga).max()


def test_autograd_iterates_match_oracle_with_schedule():
    g = synth.config0(2)["grid"]
    Y = oracle.ybus_of(g)
    S = oracle.injections(Y, g.vm, g.va)
    vm0, va0 = synth.flat_start(g)
    kw = dict(lr=1e-2, beta1=0.979, beta2=0.963, sched=1, factor=0.547, patience=5, threshold=0.0673, cooldown=3)
    r = _run(g, S, vm0[None], va0[None], kw, steps=60)
    ref = oracle.solve_adam(Y, g.bus_type, S, vm0, va0,
                            oracle.AdamOptions(tol=0.0, max_iter=60, **kw))
    assert np.abs(r["vm"][0].numpy() - ref["vm"]).max() < 1e-10
    assert np.abs(r["va"][0].numpy() - ref["va"]).max() < 1e-10
    assert r["iters"][0].item() == 60


def test_autograd_outage_matches_rebuilt_grid():
    cfg = synth.config0(3)
    g = cfg["grid"]
    Y0 = oracle.ybus_of(g)
    S = oracle.injections(Y0, g.vm, g.va)
    cand = synth.non_bridge_branches(g.n_bus, g.f, g.t)
    out = np.array([int(cand[0]), -1, int(cand[1])], dtype=np.int32)
    vm0 = np.tile(g.vm, (3, 1)) + 1e-3
    va0 = np.tile(g.va, (3, 1))
    va0[:, g.bus_type == 2] = 0.0
    r = _run(g, S, vm0, va0, dict(lr=1e-3), outage=out, steps=15)
    for c in range(3):
        Yc = oracle.ybus_of(g, skip=int(out[c]))
        ref = oracle.solve_adam(Yc, g.bus_type, S, vm0[c], va0[c], oracle.AdamOptions(lr=1e-3, tol=0.0, max_iter=15))
        assert np.abs(r["vm"][c].numpy() - ref["vm"]).max() < 1e-10
        assert np.abs(r["va"][c].numpy() - ref["va"]).max() < 1e-10
