"""Sternheimer linear response and density response (oracle; test infrastructure only).

Paper, Section 3:
  * the Sternheimer equation (h_KS - eps_v) P_c Delta psi_v = -P_c v_pert psi_v
    with P_c = 1 - P_v the projector on the conduction manifold, solved by a
    preconditioned conjugate gradient independently for every perturbation,
    spin channel and orbital;
  * the density response equation
    Delta n_j(r) = sum_sigma sum_v [psi_v^* Delta psi_jv + c.c.].

Readings taken where the paper is silent (each listed in the design doc):
  * the operator is P_c (H - eps_v) P_c on range(P_c), the right-hand side
    b = -P_c (Delta V psi_v); the unique solution lies in range(P_c);
  * preconditioner: the Teter-Payne-Allan diagonal K(x), x = T(G) / max(<psi_v|T|psi_v>, 0.1 Ha),
    applied as z = P_c K r; initial guess x = 0; maxit 1000; breakdown when
    Re<p, A p> <= 0;
  * convergence: relative 2-norm of the TRUE residual ||b - A x|| / ||b||;
  * spin-unpolarised systems carry f_s = 2 (two spin channels, equal response);
  * the chi0 block: M_ij = (Omega/N^3) sum_r dV_i(r) Dn_j(r),
    S_ij = (Omega/N^3) sum_r dV_i dV_j, eigenvalues of (sym(M), S).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import apply_H, apply_local, kinetic, to_grid
from .system import System


# ---------------------------------------------------------------- projector
def project_c(Psi: np.ndarray, y: np.ndarray) -> np.ndarray:
    """P_c y = y - sum_v psi_v <psi_v|y>   (Psi rows are the valence vectors)."""
    return y - (y @ Psi.conj().T) @ Psi


# ---------------------------------------------------------------- right-hand side
def rhs(sys: System, Psi: np.ndarray, v: int, dv_r: np.ndarray) -> np.ndarray:
    """b = -P_c (Delta V psi_v) on the sphere (Delta V applied in real space)."""
    u = apply_local(sys, dv_r, Psi[v])
    return -project_c(Psi, u)


# ---------------------------------------------------------------- direct solves
def solve_lu(H: np.ndarray, Psi: np.ndarray, eps: float, b: np.ndarray) -> np.ndarray:
    """Dense solve of P_c (H - eps) P_c x = b with b in range(P_c): the matrix
    P_c (H - eps) P_c + P_v is nonsingular and maps range(P_c) onto itself."""
    n = H.shape[0]
    Pv = Psi.T @ Psi.conj()
    Pc = np.eye(n) - Pv
    A = Pc @ (H - eps * np.eye(n)) @ Pc + Pv
    return scipy.linalg.solve(A, b)


def solve_sum_over_states(evals: np.ndarray, evecs: np.ndarray, nv: int, v: int,
                          u: np.ndarray) -> np.ndarray:
    """Delta psi_v = -sum_{c >= nv} |c> <c|u> / (eps_c - eps_v), u = Delta V psi_v
    (the first-order perturbation sum over every conduction state of H).
    ``evecs`` rows are all eigenvectors of H, ascending."""
    C = evecs[nv:]
    coef = (C.conj() @ u) / (evals[nv:] - evals[v])
    return -(coef @ C)


def free_electron_response(sys: System, val: np.ndarray, v: int, dv_r: np.ndarray) -> np.ndarray:
    """Delta psi_v of a free-electron system in closed form.

    For H = T + c (constant local potential c, no projectors) every plane wave
    is an eigenvector.  With the valence set a closed shell of plane waves
    (``val``: sphere indices of the shell, psi_v = e_{val[v]}), P_c (H - eps_v) P_c
    is diagonal on range(P_c) with entries T(G) - T(G_v), and the right-hand
    side -P_c (Delta V psi_v) has the entries -Delta V(G - G_v) (Fourier
    coefficient of the forward transform with 1/N^3) outside the shell.  The
    Sternheimer equation (Section 3) then has the solution
        Delta psi_v(G) = -Delta V(G - G_v) / (T(G) - T(G_v)),  G outside the shell,
    and 0 inside it.  The shell must be closed: every G outside it has
    T(G) > T(G_v)."""
    m = sys.miller.astype(np.int64)
    T = kinetic(sys)
    inside = np.zeros(sys.npw, bool)
    inside[val] = True
    gv = val[v]
    if not (T[~inside].min() > T[val].max()):
        raise ValueError("free_electron_response: the valence set is not a closed shell")
    dVG = np.fft.fftn(dv_r.reshape((sys.N,) * 3)) / sys.N ** 3
    d = np.mod(m - m[gv], sys.N)
    x = np.zeros(sys.npw, complex)
    out = ~inside
    x[out] = -dVG[d[out, 0], d[out, 1], d[out, 2]] / (T[out] - T[gv])
    return x


# ---------------------------------------------------------------- PCG
EKIN_FLOOR = 0.1   # Ha; keeps x finite for a band with (almost) no kinetic energy


def tpa_precond(sys: System, psi_v: np.ndarray) -> np.ndarray:
    """Teter-Payne-Allan diagonal preconditioner K(G) for band psi_v, with
    x = T(G) / max(<psi_v|T|psi_v>, 0.1 Ha)."""
    T = kinetic(sys)
    ekin = max(float(np.real(np.vdot(psi_v, T * psi_v))), EKIN_FLOOR)
    x = T / ekin
    num = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return num / (num + 16.0 * x ** 4)


def pcg_solve(sys: System, Psi: np.ndarray, eps: np.ndarray, v: int, b: np.ndarray,
              tol: float = 1e-10, maxit: int = 1000, H: np.ndarray | None = None):
    """FP64 PCG for P_c (H - eps_v) P_c x = b.  H is applied by the FFT route
    unless a dense matrix is passed.  Returns (x, iterations, true relative
    residual, status) with status 0 converged, 1 max iterations, 2 breakdown."""
    e = float(eps[v])

    def A(p):
        pc = project_c(Psi, p)
        hp = (H @ pc) if H is not None else apply_H(sys, pc)
        return project_c(Psi, hp - e * pc)

    K = tpa_precond(sys, Psi[v])
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0.0:
        return x, 0, 0.0, 0
    r = b.copy()
    z = project_c(Psi, K * r)
    p = z.copy()
    rho = float(np.real(np.vdot(r, z)))
    for it in range(1, maxit + 1):
        q = A(p)
        pq = float(np.real(np.vdot(p, q)))
        if not pq > 0.0:
            return x, it, np.linalg.norm(b - A(x)) / bn, 2
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= tol * bn:
            rt = b - A(x)
            rel = np.linalg.norm(rt) / bn
            if rel <= tol:
                return x, it, rel, 0
            r = rt                       # recursive residual drifted: restart on the true one
            z = project_c(Psi, K * r)
            p = z.copy()
            rho = float(np.real(np.vdot(r, z)))
            continue
        z = project_c(Psi, K * r)
        rho_new = float(np.real(np.vdot(r, z)))
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, maxit, np.linalg.norm(b - A(x)) / bn, 1


# ---------------------------------------------------------------- densities
def density(sys: System, Psi: np.ndarray) -> np.ndarray:
    """n(r) = (f_s / Omega) sum_v |psi_v(r)|^2 on the grid."""
    f = to_grid(sys, Psi)
    return sys.spin_factor / sys.omega * (np.abs(f) ** 2).sum(0)


def drho(sys: System, Psi: np.ndarray, dPsi: np.ndarray) -> np.ndarray:
    """Delta n(r) = f_s sum_v [psi_v^* Delta psi_v + c.c.] = (2 f_s / Omega) sum_v Re[...]."""
    a = to_grid(sys, Psi)
    d = to_grid(sys, dPsi)
    return 2.0 * sys.spin_factor / sys.omega * np.real(np.conj(a) * d).sum(0)


def chi0_block(sys: System, dv: np.ndarray, dn: np.ndarray):
    """Rayleigh-Ritz of chi0 in span{Delta V_j}: returns (eigenvalues ascending, M, S)."""
    w = sys.omega / sys.N ** 3
    A = dv.reshape(len(dv), -1)
    Bm = dn.reshape(len(dn), -1)
    M = w * (A @ Bm.T)
    S = w * (A @ A.T)
    lam = scipy.linalg.eigh(0.5 * (M + M.T), S, eigvals_only=True)
    return lam, M, S
