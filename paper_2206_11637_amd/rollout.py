"""Differentiable rollouts (reverse mode through the library's adjoint kernels)."""
from __future__ import annotations


class PFLBMRollout:  # filled in with the reverse-mode kernels
    pass


def amplitude_rollout(*args, **kwargs):
    raise NotImplementedError
