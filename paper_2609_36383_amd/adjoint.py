"""Gradients of a run's final field energy through the implicit steps, as a
torch.autograd.Function over the C ABI's adjoint calls (include/gmhc.h).

Argument marshalling and checkpoint bookkeeping only: the forward steps, the field-energy
cotangent, every adjoint step and the adjoint of initialization run in libgmhc.

Forward: load the particles (x [dim][N], or [N] in 1D; u = p/(m kappa) [3][N]; q [N]; dim 1
or 2), initialize, run
`steps` steps and return W(T), saving a checkpoint image of the accepted state every
`every` steps.  Backward: from dW/d(state) at T, walk the checkpoint segments from last
to first; each segment is re-run from its checkpoint (bitwise the same steps with
deterministic = 1), keeping the image of every state and the converged current and orbit
velocities of every step, and the steps are then reversed one by one with
gmhc_adjoint_step; at the first state gmhc_adjoint_initialize maps the cotangents to the
loaded inputs.  The charge cotangent sums every step's part and initialization's.
"""
import time

import numpy as np
import torch

from . import gmhc as G


class FieldEnergyRun(torch.autograd.Function):
    """W(T) = FieldEnergyRun.apply(x, u, q, cfg, steps, every, device, potentials)."""

    @staticmethod
    def forward(ctx, x, u, q, cfg, steps, every, device, potentials=None):
        n = int(q.numel())
        sim = G.Simulation(cfg, n, device=device)
        sim.load_particles(x.detach().cpu().numpy(), u.detach().cpu().numpy(), q.detach().cpu().numpy())
        if potentials is not None:
            sim.load_potentials(*potentials)
        sim.initialize()
        nbytes = sim.state_bytes()
        ckpt = {}

        def save():
            img = torch.empty(nbytes, dtype=torch.uint8, device=sim.device)
            sim.save(img)
            return img

        ckpt[0] = save()
        for k in range(steps):
            sim.step()
            if (k + 1) % every == 0 and k + 1 < steps:
                ckpt[k + 1] = save()
        W = sim.diagnostics()["field"]
        ctx.sim, ctx.ckpt, ctx.steps, ctx.every, ctx.save_fn = sim, ckpt, steps, every, save
        ctx.devices = (x.device, u.device, q.device)
        ctx.xshape = x.shape
        ctx.reports = []
        ctx.seconds = {"rerun": 0.0, "adjoint_steps": 0.0}
        return torch.tensor(W, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gW):
        sim, steps = ctx.sim, ctx.steps
        dev = sim.device
        n, ng, d = sim.np, sim.ng, sim.d
        f64 = dict(dtype=torch.float64, device=dev)
        scratch = sim.adjoint_scratch()
        lf = torch.empty(9, ng, **f64)
        sim.energy_grad(lf)
        lf *= float(gW)
        lx = torch.zeros(d, n, **f64)
        lP = torch.zeros(3, n, **f64)
        gq = torch.zeros(n, **f64)
        gq_step = torch.empty(n, **f64)
        starts = sorted(ctx.ckpt)
        for a in reversed(starts):
            b = min(a + ctx.every, steps)
            t0 = time.perf_counter()
            sim.load(ctx.ckpt[a])
            images, js, vbars = [], [], []
            for _ in range(a, b):
                images.append(ctx.save_fn())
                sim.step()
                j = torch.empty(3, ng, **f64)
                vb = torch.empty(3, n, **f64)
                sim.read_field_into("J", j)
                sim.read_particles_into(vbar=vb)
                js.append(j)
                vbars.append(vb)
            torch.cuda.synchronize(dev)
            t1 = time.perf_counter()
            ctx.seconds["rerun"] += t1 - t0
            for k in reversed(range(len(images))):
                sim.load(images[k])
                rep = sim.adjoint_step(scratch, js[k], vbars[k], lx, lP, lf, lx, lP, gq_step, lf)
                ctx.reports.append(rep)
                gq += gq_step
            ctx.seconds["adjoint_steps"] += time.perf_counter() - t1
        sim.load(ctx.ckpt[0])
        gx = torch.empty(d, n, **f64)
        gu = torch.empty(3, n, **f64)
        sim.adjoint_initialize(scratch, lx, lP, lf, gx, gu, gq_step)
        gq += gq_step
        torch.cuda.synchronize(dev)
        dx, du, dq = ctx.devices
        return gx.reshape(ctx.xshape).to(dx), gu.to(du), gq.to(dq), None, None, None, None, None


def field_energy_run(x, u, q, cfg, steps, every=10, device="cuda", potentials=None):
    """W(T) after `steps` steps from the particles (x [dim][N] or [N] in 1D, u [3][N], q [N],
    float64 torch tensors, any device), differentiable with respect to x, u and q.  potentials: optional
    initial (A0, U0) [3][Ng] arrays, held fixed."""
    return FieldEnergyRun.apply(x, u, q, cfg, int(steps), int(every), device, potentials)


def quiet1d_inputs(w, eps, u0, device="cpu"):
    """The particles of a "quiet1d" workload as torch functions of its perturbation
    amplitudes eps [nmodes] and beam momentum u0 (workloads.quiet1d_parts)."""
    from . import workloads as W
    xj, pat = W.quiet1d_parts(w)
    L = w["length"][0]
    nb = xj.size
    pat_t = torch.as_tensor(pat, dtype=torch.float64, device=device)
    wgt = 0.5 * (L / nb) * (1.0 + eps @ pat_t)
    q = -torch.cat([wgt, wgt])
    x = torch.as_tensor(np.concatenate([xj, xj]), dtype=torch.float64, device=device)
    ux = torch.cat([u0 * torch.ones(nb, dtype=torch.float64, device=device),
                    -u0 * torch.ones(nb, dtype=torch.float64, device=device)])
    z = torch.zeros(2 * nb, dtype=torch.float64, device=device)
    u = torch.stack([ux, z, z])
    return x, u, q
