"""The online least-squares problem of eq. elliptic_cond_reduced on an
ill-conditioned system: why the library takes a corrected semi-normal step.

The paper writes the least-squares gluing through its normal equations.  On
the high-contrast medium of Sec. 5.2 (contrast 1e3) with full bases on 4 x 4
patches at h = 1/64, kappa(P~) is about 1e6: the normal equations (Cholesky of
P~^T P~ in FP64) leave the reconstruction about 2e-6 from the fine solution
(their error bound is about kappa^2 u), one step of the corrected semi-normal
equations (Bjorck: r = d - P~ c, then the normal equations for the correction
with the same factor) about 3e-11, the accuracy of the oracle's Householder QR.  The system is consistent (full bases reproduce
the fine solution), so the brute-force fine solve is the reference for the
reconstructed solutions.
"""
import numpy as np
import scipy.linalg as sla

import synth
from oracle import elliptic as E


def test_corrected_semi_normal_step_reaches_qr_accuracy():
    N, M = 64, 4
    a = synth.high_contrast_coefficient(N, 1000.0)
    ref = E.offline(a, N, M, np.full(M * M, 8, dtype=np.int32), 8, 8, full_basis=True)
    P, n_cont, drows, off = E.coarse_rows(N, M, ref, a)
    phi = synth.dirichlet_sin_cos(N)
    d = np.zeros(P.shape[0])
    d[n_cont:] = phi[drows]
    kappa = np.linalg.cond(P)
    assert 1e5 < kappa < 1e7, kappa
    K = P.T @ P
    L = np.linalg.cholesky(K)

    def solve(b):
        return sla.solve_triangular(L.T, sla.solve_triangular(L, b, lower=True), lower=False)

    c_ne = solve(P.T @ d)
    c_csne = c_ne + solve(P.T @ (d - P @ c_ne))
    Qf, Rf = E.coarse_factor(P)
    c_qr = E.coarse_solve(Qf, Rf, n_cont, drows, phi)[:, 0]
    u_fine = E.global_solve(a, N, phi)
    err = {name: E.relative_l2(E.reconstruct(N, M, ref, off, c)[:, 0], u_fine)
           for name, c in (("ne", c_ne), ("csne", c_csne), ("qr", c_qr))}
    # QR and the corrected step: about kappa u; the normal equations alone: about kappa^2 u
    assert err["qr"] < 1e-9 and err["csne"] < 1e-9, err
    assert err["ne"] > 1e-8 and err["ne"] > 100 * err["csne"], err
    assert np.linalg.norm(c_csne - c_qr) / np.linalg.norm(c_qr) < 1e-9
