"""Named synthetic workloads (sizes, seeds, readings of unstated parameters).

Each workload is a plain dict; the coefficient field and the overlaps are
drawn by the generators in :mod:`synth` from the seeds stated here.
"""
from __future__ import annotations

import numpy as np

from . import (lognormal_coefficient, overlap_draw, periodic_coefficient,
               dirichlet_sin_cos, kinetic_sigma, two_scale_coefficient, high_contrast_coefficient,
               dirichlet_sine)

COEF_SEED = 1
OMEGA_SEED = 2
OVERLAP_SEED = 3
REQUEST_SEED = 4
ARRIVAL_SEED = 5


def elliptic_periodic_128():
    """h=1/128, 4x4 patches, overlap 8 cells, 10 samples, rank 6, periodic medium eps=1/16."""
    N, M = 128, 4
    return dict(name="elliptic_periodic_N128_M4_s10_k6", kind="elliptic", N=N, M=M,
                overlap=np.full(M * M, 8, dtype=np.int32), s=10, k=6,
                coef=periodic_coefficient(N, 1.0 / 16.0), phi=dirichlet_sin_cos(N),
                seed=OMEGA_SEED)


def elliptic_lognormal_512():
    """h=1/512, 8x8 patches, overlap 16 cells, 32 samples, rank 12, lognormal medium ell=1/64."""
    N, M = 512, 8
    return dict(name="elliptic_lognormal_N512_M8_s32_k12", kind="elliptic", N=N, M=M,
                overlap=np.full(M * M, 16, dtype=np.int32), s=32, k=12,
                coef=lognormal_coefficient(N, 1.0 / 64.0, COEF_SEED), phi=dirichlet_sin_cos(N),
                seed=OMEGA_SEED)


def elliptic_lognormal_1024():
    """h=1/1024, 16x16 patches, overlap per patch from {16, 32} cells, 64 samples, rank 16, ell=1/128."""
    N, M = 1024, 16
    return dict(name="elliptic_lognormal_N1024_M16_s64_k16", kind="elliptic", N=N, M=M,
                overlap=overlap_draw(M, (16, 32), OVERLAP_SEED), s=64, k=16,
                coef=lognormal_coefficient(N, 1.0 / 128.0, COEF_SEED), phi=dirichlet_sin_cos(N),
                seed=OMEGA_SEED)


def kinetic_slab_4096():
    """1D slab, 4096 cells, 32 Gauss-Legendre ordinates, 32 patches, buffer 64 cells, 48 samples, rank 10."""
    Nx, M = 4096, 32
    return dict(name="kinetic_slab_Nx4096_M32_s48_k10", kind="kinetic", N=Nx, M=M,
                overlap=np.full(M, 64, dtype=np.int32), s=48, k=10, n_vel=32, eps=2.0 ** -8,
                coef=kinetic_sigma(Nx), seed=OMEGA_SEED)


def elliptic_two_scale_100(k=10):
    """The paper's elliptic test: h=1/100, 5x5 patches of 20x20 cells, buffered
    patches concentric with all sides twice as long (10 cells, clipped at the
    domain), k random samples and rank k (the paper's k_m, no oversampling),
    two-scale medium eps=2^-4, sine boundary data."""
    N, M = 100, 5
    return dict(name=f"elliptic_two_scale_N100_M5_k{k}", kind="elliptic", N=N, M=M,
                overlap=np.full(M * M, 10, dtype=np.int32), s=k, k=k,
                coef=two_scale_coefficient(N, 2.0 ** -4), phi=dirichlet_sine(N), seed=OMEGA_SEED)


def elliptic_high_contrast_100(k=6):
    """The paper's high-contrast comparison: h=1/100, 5x5 patches (H=1/5), the
    same buffers as the two-scale test, k random samples and rank k."""
    N, M = 100, 5
    return dict(name=f"elliptic_high_contrast_N100_M5_k{k}", kind="elliptic", N=N, M=M,
                overlap=np.full(M * M, 10, dtype=np.int32), s=k, k=k,
                coef=high_contrast_coefficient(N), phi=dirichlet_sine(N), seed=OMEGA_SEED)


def kinetic_hg_100(eps=2.0 ** -6, k=10, n_vel=64):
    """The paper's transport test (Sec. 4.3): dx=0.01 (100 cells), M=10, buffered
    patches twice as large (5 cells each side), Henyey-Greenstein scattering
    with g=1/2 and sigma=1, k random samples and rank k, full bases on the two
    end patches; 64 Gauss-Legendre ordinates stand in for the paper's 120-point
    grid (the end patches' full basis has one column per ordinate, at most 64)."""
    Nx, M = 100, 10
    return dict(name=f"kinetic_hg_Nx100_M10_k{k}_eps{eps:g}", kind="kinetic", N=Nx, M=M,
                overlap=np.full(M, 5, dtype=np.int32), s=k, k=k, n_vel=n_vel, eps=eps, hg=0.5,
                coef=np.ones(Nx), seed=OMEGA_SEED)


def small_elliptic(N=32, M=2, delta=4, s=8, k=5, coef="periodic"):
    """Small elliptic case for fast parity tests (several tiles, ragged sizes)."""
    if coef == "periodic":
        a = periodic_coefficient(N, 1.0 / 8.0)
    else:
        a = lognormal_coefficient(N, 4.0 / N, COEF_SEED)
    return dict(name=f"elliptic_small_N{N}_M{M}", kind="elliptic", N=N, M=M,
                overlap=np.full(M * M, delta, dtype=np.int32), s=s, k=k, coef=a,
                phi=dirichlet_sin_cos(N), seed=OMEGA_SEED)


WORKLOADS = {
    "elliptic_periodic_128": elliptic_periodic_128,
    "elliptic_lognormal_512": elliptic_lognormal_512,
    "elliptic_lognormal_1024": elliptic_lognormal_1024,
    "kinetic_slab_4096": kinetic_slab_4096,
    "elliptic_two_scale_100": elliptic_two_scale_100,
    "elliptic_high_contrast_100": elliptic_high_contrast_100,
    "kinetic_hg_100": kinetic_hg_100,
}
