"""Hutchinson estimate of diag(K⁻¹) (TEST INFRASTRUCTURE).

For Rademacher probes z (entries ±1 with equal probability), E[z ∘ K⁻¹z] = diag(K⁻¹) because
E[z zᵀ] = I. With s probes the estimate is ĥ = (1/s) Σ_k z_k ∘ (K⁻¹ z_k). Averaging over all 2ⁿ
sign vectors makes the off-diagonal terms cancel exactly, so that average equals diag(K⁻¹).
For SPD K, (K⁻¹)_ii ≥ 1/K_ii (Cauchy–Schwarz on e_iᵀK^{1/2}·K^{-1/2}e_i), which is the clamp used
for training targets.
"""
from __future__ import annotations

import itertools

import numpy as np


def estimate(solve, probes):
    """probes: s×n array of ±1; solve(v) returns K⁻¹v. Returns ĥ (n)."""
    probes = np.asarray(probes, dtype=np.float64)
    acc = np.zeros(probes.shape[1])
    for z in probes:
        acc += z * solve(z)
    return acc / probes.shape[0]


def all_sign_vectors(n):
    return np.array(list(itertools.product((-1.0, 1.0), repeat=n)))


def clamp_targets(h, Kdiag):
    return np.maximum(h, 1.0 / np.asarray(Kdiag))
