"""Linear (von Neumann) theory of the scheme, used to pin the oracle.

Two models: the paper's forcing model (Eq. 5, model=0) below, and the
altered-equilibrium model (model=1) of the oracle's lbmref_equilibrium_c2,
whose linearised equilibrium is feq_i ~ w_i (3 c^2 drho + 3 e_i.j) for
i != 0 and feq_0 ~ (1 - 5 c^2 / 3) drho (what is left of drho), with no
source term.

Written from the paper's equations independently of the oracle: around rest
(rho = 1, u = 0) a perturbation delta f_i(x) = a_i exp(i k.x) obeys
  a(t+1) = M(k) a(t),
  M(k) = diag(exp(-i k.e_i)) [ I - (I - J)/tau + A(k) ],
where J_ij = w_i (1 + 3 e_i.e_j) is the linearised equilibrium of Eq. 2
(feq_i ~ w_i (drho + 3 e_i.j)), A(k)_ij = 3 w_i alpha i (e_ix sin k_x +
e_iy sin k_y) is the source of Eq. 5 with the central difference
(rho(x+1) - rho(x-1))/2 -> i sin(k) rho_hat, and the diagonal factor is the
streaming f_i(x + e_i, t + 1) = f*_i(x, t).
"""
import numpy as np

# Link vectors and weights, evaluated by hand from the formulas of Sec. 2.
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
              [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def matrix(kx, ky, tau, c2, model=0):
    if model == 1:
        J = W[:, None] * (3.0 * c2 + 3.0 * (E @ E.T))
        J[0, :] = 1.0 - 5.0 * c2 / 3.0
        A = np.zeros((9, 9), dtype=complex)
    else:
        alpha = 1.0 / 3.0 - c2
        J = W[:, None] * (1.0 + 3.0 * (E @ E.T))
        A = 3.0 * W[:, None] * alpha * 1j * (E[:, 0] * np.sin(kx) + E[:, 1] * np.sin(ky))[:, None] * np.ones((1, 9))
    C = np.eye(9) - (np.eye(9) - J) / tau + A
    S = np.diag(np.exp(-1j * (E[:, 0] * kx + E[:, 1] * ky)))
    return S @ C


def evolve_fields(amp_rho, kx, ky, nx, ny, tau, c2, t, amp_u=(0.0, 0.0), model=0):
    """Linear prediction of (drho, jx, jy) on an nx x ny grid after t steps for
    the initial state f = feq(1 + amp_rho sin(k.x), u = amp_u sin(k.x))."""
    # sin(k.x) = (exp(ik.x) - exp(-ik.x)) / (2i); feq linearised: w_i(drho + 3 e_i.u)
    ej = E[:, 0] * amp_u[0] + E[:, 1] * amp_u[1]
    if model == 1:
        a0 = W * (3.0 * c2 * amp_rho + 3.0 * ej)
        a0[0] = (1.0 - 5.0 * c2 / 3.0) * amp_rho
        a0 = a0 / 2j
    else:
        a0 = W * (amp_rho + 3.0 * ej) / 2j
    M = matrix(kx, ky, tau, c2, model)
    a = np.linalg.matrix_power(M, t) @ a0
    y, x = np.mgrid[0:ny, 0:nx]
    ph = np.exp(1j * (kx * x + ky * y))
    rho = 2.0 * np.real(a.sum() * ph)
    jx = 2.0 * np.real((a * E[:, 0]).sum() * ph)
    jy = 2.0 * np.real((a * E[:, 1]).sum() * ph)
    return rho, jx, jy


def acoustic_eigs(kx, ky, tau, c2, model=0):
    """The three eigenvalues of M(k) of largest modulus: the two sound modes
    and the shear mode (which of them decays slowest depends on c2)."""
    lam = np.linalg.eigvals(matrix(kx, ky, tau, c2, model))
    order = np.argsort(-np.abs(lam))
    return lam[order[:3]]


def spectral_radius(kx, ky, tau, c2, model=0):
    return np.max(np.abs(np.linalg.eigvals(matrix(kx, ky, tau, c2, model))))
