"""Differentiable rollouts through the library's reverse-mode kernels.

PFLBMRollout maps (phi0, M, sigma, xi) to the interface-amplitude trace
    a(n) = < sum_y phi^n(x0, y, z) >_z - depth ,   n = K, 2K, ..., N
(the column-sum elevation probe of the paper's standing-wave tests, sec.
"Gravity wave" setup).  Its backward runs the adjoint step kernels in reverse
time, with sqrt(N) checkpointing: the forward keeps every S-th state
(S ~ sqrt(N)); the backward recomputes each checkpoint's segment of S states
out of place (state k+1 written straight from state k into the segment
buffer, no copies) and walks it backwards.  Peak memory is about 2 sqrt(N)
saved states instead of N.  The recompute is bit-identical to the original
forward (deterministic kernels).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

from . import _lib


@dataclasses.dataclass
class RolloutSpec:
    sim: object                 # paper_2206_11637_amd.sim.Simulation
    params: object              # base parameters (M and sigma are overridden)
    nsteps: int
    sample_every: int
    depth: float
    x0: int = 0
    u0: Optional[torch.Tensor] = None
    pstar0: Optional[torch.Tensor] = None
    checkpoint_every: Optional[int] = None
    stats: dict = dataclasses.field(default_factory=dict)


def _params_with(p, M, sigma, xi):
    if isinstance(p, dict):
        q = dict(p)
        q["mobility"], q["sigma"], q["xi"] = M, sigma, xi
        return q
    return dataclasses.replace(p, mobility=M, sigma=sigma, xi=xi)


def _amplitude(sim, x0, depth):
    phi = sim.phi()                                  # [nz, ny, nx] float64
    return phi[:, :, x0].sum(dim=1).mean() - depth


class PFLBMRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, M, sigma, xi, spec: RolloutSpec):
        sim = spec.sim
        N, K = spec.nsteps, spec.sample_every
        S = spec.checkpoint_every or max(1, int(math.ceil(math.sqrt(N))))
        sim.set_params(_params_with(spec.params, float(M), float(sigma), float(xi)))
        sim.init_equilibrium(phi0.detach(), spec.u0, spec.pstar0)
        ckpt = {0: sim.save_state()}
        trace = []
        n = 0
        while n < N:
            # advance to the next sample or checkpoint boundary
            nxt = min(N, (n // K + 1) * K, (n // S + 1) * S)
            sim.step(nxt - n)
            n = nxt
            if n % K == 0:
                trace.append(_amplitude(sim, spec.x0, spec.depth))
            if n % S == 0 and n < N:
                ckpt[n] = sim.save_state()
        ctx.spec = spec
        ctx.ckpt = ckpt
        ctx.S = S
        ctx.M, ctx.sigma, ctx.xi = float(M), float(sigma), float(xi)
        spec.stats["checkpoints"] = len(ckpt)
        spec.stats["checkpoint_every"] = S
        return torch.stack(trace)

    @staticmethod
    def backward(ctx, grad_trace):
        spec, ckpt, S = ctx.spec, ctx.ckpt, ctx.S
        sim = spec.sim
        N, K = spec.nsteps, spec.sample_every
        nz, ny, nx = sim.shape
        grad_trace = grad_trace.detach().to(device=sim.device, dtype=torch.float64)
        sim.set_params(_params_with(spec.params, ctx.M, ctx.sigma, ctx.xi))
        sim.adjoint_attach()
        sim.adjoint_reset()
        inj = torch.zeros(sim.shape, dtype=torch.float64, device=sim.device)

        def inject(level):
            if level > 0 and level % K == 0:
                inj[:, :, spec.x0] = grad_trace[level // K - 1] / nz
                sim.adjoint_inject_phi(inj)

        # segment buffer: slot 0 is the checkpoint itself, slots 1..S-1 are
        # recomputed out of place from the previous slot (no state copies)
        seg = torch.empty((max(S - 1, 1), sim.state_bytes()), dtype=torch.uint8, device=sim.device)
        # two-buffer contexts chain the recompute: each step writes the phase
        # field it forms into the state it read and leaves the next state's to
        # the following step (the last step of a segment forms it itself)
        chain = getattr(sim, "streaming", "ab") == "ab"
        starts = sorted(ckpt)
        for a in reversed(starts):
            b = min(a + S, N)
            states = [ckpt[a]]
            for n in range(a, b - 1):
                flags = 0
                if chain:
                    flags = _lib.STATES_WRITE_SRC_PHI
                    if n < b - 2:
                        flags |= _lib.STATES_SKIP_DST_PHI
                sim.step_states(states[-1], seg[n - a], n, flags)
                states.append(seg[n - a])
            for n in range(b - 1, a - 1, -1):
                inject(n + 1)
                sim.adjoint_step(states[n - a], n)
        dphi0 = sim.adjoint_init(spec.u0)
        dM, dsig, dxi = sim.adjoint_grads()
        spec.stats["segment_states"] = S
        dev = grad_trace.device
        return (dphi0.reshape(nz, ny, nx), torch.tensor(dM, dtype=torch.float64, device=dev),
                torch.tensor(dsig, dtype=torch.float64, device=dev),
                torch.tensor(dxi, dtype=torch.float64, device=dev), None)


def amplitude_rollout(sim, phi0, M, sigma, *, params, nsteps, sample_every, depth, x0=0,
                      u0=None, pstar0=None, checkpoint_every=None, stats=None, xi=None):
    """Differentiable amplitude trace (see module docstring).  phi0 is a
    float64 tensor [nz, ny, nx] on the simulation's device; M, sigma and xi
    (default: the interface width of params, held fixed) are 0-dim float64
    tensors.  dL/dxi holds phi0 fixed; a phi0 computed from xi in torch adds
    its own term through dL/dphi0.  Returns a float64 tensor of
    nsteps // sample_every samples."""
    if xi is None:
        xi = torch.tensor(float(params["xi"] if isinstance(params, dict) else params.xi),
                          dtype=torch.float64)
    spec = RolloutSpec(sim, params, nsteps, sample_every, depth, x0,
                       None if u0 is None else torch.as_tensor(u0, dtype=torch.float64).to(sim.device),
                       None if pstar0 is None else torch.as_tensor(pstar0, dtype=torch.float64).to(sim.device),
                       checkpoint_every, stats if stats is not None else {})
    return PFLBMRollout.apply(phi0, M, sigma, xi, spec)
