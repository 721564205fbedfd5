"""Shared test helpers: seeded workloads, the per-site error metric, and
canonical even-odd field helpers.  No operator arithmetic lives here."""

from __future__ import annotations

import functools

import numpy as np

import fieldgen

THETA_AP = (1.0, 0.0, 0.0, 0.0)   # antiperiodic in time

# Workloads: 8^4 single hop (kappa 0.16); 32^3x64 Qtm + CG (kappa 0.1632,
# 2 kappa mu = 0.0013); 48^3x96 smoothed links for mixed precision; 24^3x48
# adjoint.
HOP8 = dict(dims=(8, 8, 8, 8), kappa=0.16, seed=fieldgen.SEEDS["hop8"])
QTM32 = dict(dims=(64, 32, 32, 32), kappa=0.1632, mt=0.0013, seed=fieldgen.SEEDS["qtm32"])


def mu_of(kappa, mt):
    """Bare twisted mass from 2 kappa mu."""
    return mt / (2.0 * kappa)


def site_rel_err(out, ref):
    """max over sites of |out(x) - ref(x)|_2 / max(|ref(x)|_2, 1e-6 rms_site)."""
    out = np.asarray(out).reshape(len(ref), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    num = np.linalg.norm(out - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    rms = np.sqrt(np.mean(den ** 2)) if len(den) else 0.0
    den = np.maximum(den, 1e-6 * rms)
    den[den == 0] = 1.0
    return float(np.max(num / den)) if len(num) else 0.0


@functools.lru_cache(maxsize=4)
def haar(dims, seed):
    return fieldgen.gauge_haar(dims, seed)


@functools.lru_cache(maxsize=8)
def gauss(n, seed):
    return fieldgen.spinor_gauss(n, seed)


def round_f32(a):
    """FP32-rounded copy of a complex128 field (what the FP32 path is fed)."""
    return a.astype(np.complex64).astype(np.complex128)
