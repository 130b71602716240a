"""Plain PyTorch autograd DPF: the comparison system for the fused adjoint.

This is Algorithm 1 as the paper implements it -- the forward pass in torch
ops on a sparse CSR admittance matrix, ``loss.backward()`` for the gradient,
an Adam step -- run on the same GPU, inputs and stopping rule as
dpf_solve_batch so that the two compute the same iterates.  Differences from
the paper's loop that keep the comparison fair: every case has its own loss,
Adam step count, learning-rate schedule and stop test (a converged case is
frozen, the batch keeps running until all are done or the cap is hit), and the
stop test is evaluated on the host only every ``poll`` iterations.

Y is split into real CSR matrices G and B (I = (G + jB)(Vr + jVi)) because
float64 CSR products are the sparse kernels torch supports on every backend.
It is never used by the product path; it only runs inside bench.py and tests.
"""

from __future__ import annotations

import math

import torch

from .binding import PQ, PV, SLACK, Options, SCHED_PLATEAU, SCHED_STEP


class AutogradDPF:
    def __init__(self, row_ptr, col, val, n_bus, bus_type, s_spec, outage=None, branch=None, device="cuda"):
        """row_ptr/col/val: CSR of Y (val complex128); bus_type [n]; s_spec [n] or [B, n]
        complex; outage [B] branch index or -1; branch = (f, t, r, x, b) arrays."""
        dev = torch.device(device)
        rp = torch.as_tensor(row_ptr, dtype=torch.int64, device=dev)
        ci = torch.as_tensor(col, dtype=torch.int64, device=dev)
        v = torch.as_tensor(val, dtype=torch.complex128, device=dev)
        self.n = n_bus
        self.G = torch.sparse_csr_tensor(rp, ci, v.real.contiguous(), (n_bus, n_bus))
        self.Bm = torch.sparse_csr_tensor(rp, ci, v.imag.contiguous(), (n_bus, n_bus))
        bt = torch.as_tensor(bus_type, device=dev)
        self.wP = (bt != SLACK).to(torch.float64)
        self.wQ = (bt == PQ).to(torch.float64)
        self.learn_vm = (bt == PQ).to(torch.float64)
        self.learn_va = (bt != SLACK).to(torch.float64)
        self.m = float(self.wP.sum() + self.wQ.sum())
        s = torch.as_tensor(s_spec, dtype=torch.complex128, device=dev)
        self.Sr = s.real.contiguous()
        self.Si = s.imag.contiguous()
        self.outage = None
        if outage is not None:
            f, t, r, x, b = (torch.as_tensor(a, device=dev) for a in branch)
            out = torch.as_tensor(outage, dtype=torch.int64, device=dev)
            has = out >= 0
            k = torch.where(has, out, torch.zeros_like(out))
            d = r[k] ** 2 + x[k] ** 2
            yr, yi = r[k] / d, -x[k] / d
            mask = has.to(torch.float64)
            self.outage = (f[k].long(), t[k].long(), yr * mask, yi * mask, 0.5 * b[k] * mask)

    def _current(self, Vr, Vi):
        # [B, n] -> [B, n] with the CSR product on the transposed dense block
        Ir = (torch.sparse.mm(self.G, Vr.T) - torch.sparse.mm(self.Bm, Vi.T)).T
        Ii = (torch.sparse.mm(self.G, Vi.T) + torch.sparse.mm(self.Bm, Vr.T)).T
        if self.outage is not None:
            f, t, yr, yi, bh = self.outage
            ar = torch.arange(Vr.shape[0], device=Vr.device)
            vfr, vfi, vtr, vti = Vr[ar, f], Vi[ar, f], Vr[ar, t], Vi[ar, t]
            # rank-2 block [[y + j b/2, -y], [-y, y + j b/2]] on (f, t)
            dfr = yr * (vfr - vtr) - yi * (vfi - vti) - bh * vfi
            dfi = yr * (vfi - vti) + yi * (vfr - vtr) + bh * vfr
            dtr = yr * (vtr - vfr) - yi * (vti - vfi) - bh * vti
            dti = yr * (vti - vfi) + yi * (vtr - vfr) + bh * vtr
            Ir = Ir.index_put((ar, f), -dfr, accumulate=True).index_put((ar, t), -dtr, accumulate=True)
            Ii = Ii.index_put((ar, f), -dfi, accumulate=True).index_put((ar, t), -dti, accumulate=True)
        return Ir, Ii

    def loss(self, vm, va):
        """Per-case MSE loss [B] and max |residual| [B] (differentiable in vm, va)."""
        Vr = vm * torch.cos(va)
        Vi = vm * torch.sin(va)
        Ir, Ii = self._current(Vr, Vi)
        # S = V conj(I)
        Pc = Vr * Ir + Vi * Ii
        Qc = Vi * Ir - Vr * Ii
        rP = (Pc - self.Sr) * self.wP
        rQ = (Qc - self.Si) * self.wQ
        loss = (rP * rP + rQ * rQ).sum(dim=1) / self.m
        mu = torch.maximum(rP.abs().amax(dim=1), rQ.abs().amax(dim=1))
        return loss, mu

    def solve(self, vm0, va0, opts: Options, poll: int = 1, max_iter=None, time_only_iters=None,
              time_budget_s=None):
        """Run the iteration; returns dict like dpf.solve plus the final vm, va,
        the number of loop passes and whether the time budget ended the run.

        time_only_iters: run exactly that many iterations without stop tests
        (for per-iteration timing).  time_budget_s: at each host poll, stop once
        this much wall time has passed (cases still running keep status 1)."""
        import time as _time

        t_start = _time.perf_counter()
        budget_hit = False
        vm = vm0.clone().requires_grad_(True)
        va = va0.clone().requires_grad_(True)
        Bc = vm.shape[0]
        dev = vm.device
        mv = torch.zeros_like(vm)
        ma = torch.zeros_like(va)
        sv = torch.zeros_like(vm)
        sa = torch.zeros_like(va)
        t = torch.zeros(Bc, dtype=torch.float64, device=dev)
        lr = torch.full((Bc,), opts.lr, dtype=torch.float64, device=dev)
        best = torch.full((Bc,), math.inf, dtype=torch.float64, device=dev)
        bad = torch.zeros(Bc, dtype=torch.int64, device=dev)
        cool = torch.zeros(Bc, dtype=torch.int64, device=dev)
        active = torch.ones(Bc, dtype=torch.bool, device=dev)
        status = torch.ones(Bc, dtype=torch.int32, device=dev)
        iters = torch.zeros(Bc, dtype=torch.int32, device=dev)
        mu_out = torch.zeros(Bc, dtype=torch.float64, device=dev)
        cap = opts.max_iter if max_iter is None else max_iter
        n_run = cap if time_only_iters is None else time_only_iters
        for it in range(n_run + 1):
            loss, mu = self.loss(vm, va)
            with torch.no_grad():
                if time_only_iters is None:
                    nonfin = active & ~(torch.isfinite(loss) & torch.isfinite(mu))
                    conv = active & ~nonfin & (mu < opts.tol)
                    status = torch.where(nonfin, torch.full_like(status, 2), status)
                    status = torch.where(conv, torch.zeros_like(status), status)
                    mu_out = torch.where(active, mu, mu_out)
                    active = active & ~nonfin & ~conv
                    if it == n_run:
                        break
                    if it % poll == 0:
                        if not bool(active.any()):
                            break
                        if time_budget_s is not None and _time.perf_counter() - t_start > time_budget_s:
                            budget_hit = True
                            break
                elif it == n_run:
                    break
            gvm, gva = torch.autograd.grad(loss.sum(), (vm, va))
            with torch.no_grad():
                a = active.to(torch.float64)[:, None]
                t = t + active.to(torch.float64)
                bc1 = (1.0 - opts.beta1 ** t)[:, None]
                bc2 = (1.0 - opts.beta2 ** t)[:, None]
                bc1 = torch.where(bc1 > 0, bc1, torch.ones_like(bc1))
                bc2 = torch.where(bc2 > 0, bc2, torch.ones_like(bc2))
                for x, m_, s_, g, lm in ((vm, mv, sv, gvm, self.learn_vm), (va, ma, sa, gva, self.learn_va)):
                    upd = a * lm
                    m_.copy_(torch.where(upd > 0, opts.beta1 * m_ + (1 - opts.beta1) * g, m_))
                    s_.copy_(torch.where(upd > 0, opts.beta2 * s_ + (1 - opts.beta2) * g * g, s_))
                    step = lr[:, None] * (m_ / bc1) / (torch.sqrt(s_ / bc2) + opts.eps)
                    x.sub_(torch.where(upd > 0, step, torch.zeros_like(step)))
                iters = iters + active.to(torch.int32)
                if opts.sched == SCHED_PLATEAU:
                    imp = loss < best * (1.0 - opts.threshold)
                    best = torch.where(active & imp, loss, best)
                    bad = torch.where(active, torch.where(imp, torch.zeros_like(bad), bad + 1), bad)
                    incd = active & (cool > 0)
                    cool = torch.where(incd, cool - 1, cool)
                    bad = torch.where(incd, torch.zeros_like(bad), bad)
                    red = active & (bad > opts.patience)
                    nl = torch.clamp(lr * opts.factor, min=opts.min_lr)
                    lr = torch.where(red & (lr - nl > opts.sched_eps), nl, lr)
                    cool = torch.where(red, torch.full_like(cool, opts.cooldown), cool)
                    bad = torch.where(red, torch.zeros_like(bad), bad)
                elif opts.sched == SCHED_STEP and opts.patience > 0:
                    # StepLR on the case's step count t (the solve starts at t = 0)
                    stepped = active & ((t.long() % opts.patience) == 0)
                    lr = torch.where(stepped, lr * opts.factor, lr)
        return {"vm": vm.detach(), "va": va.detach(), "status": status, "iters": iters, "max_mis": mu_out,
                "loops": it, "budget_hit": budget_hit}
