"""Independent checks of the oracle: a dense Newton solve of the whole
backward-Euler system and a stand-alone Bose-Einstein intensity.

Nothing here is shared with the oracle or with the GPU library.  The
formulation is deliberately different from the oracle's: face fluxes are
assembled in conservative form over *all* faces (outflow with the cell value,
inflow with the neighbour or wall ghost, Eq. eq-bte-fv with the ghosts of
Eq. eq-bdry), the equilibrium derivative is taken by complex-step
differentiation, and mirror maps are found by a nearest-vector search.  The
unknowns are every intensity I[P, d, b] plus every cell temperature T[P]; the
equations are the implicit finite-volume balances plus, per cell, the
energy-consistency relation that defines T (relaxation-time weighted, or the
plain energy sum).
"""
from __future__ import annotations

import numpy as np

HBAR = 1.054571817e-34
KB = 1.380649e-23


def planck_coeff(inst):
    """Per-band prefactor of the equilibrium intensity per steradian:
    (modes per volume in the band) x hbar omega / (4 pi)."""
    return inst.deg * inst.dos * inst.domega * HBAR * inst.omega / (4.0 * np.pi)


def equilibrium(inst, T):
    """Bose-Einstein equilibrium intensity, array [..., N_b] for T of any shape."""
    T = np.asarray(T)[..., None]
    x = HBAR * inst.omega / (KB * T)
    return planck_coeff(inst) / np.expm1(x)


def _mirror(s, axis):
    t = s.copy()
    t[:, axis] = -t[:, axis]
    dist = np.abs(s[None, :, :] - t[:, None, :]).max(axis=2)
    m = dist.argmin(axis=1)
    assert np.all(dist[np.arange(len(m)), m] < 1e-10), "direction set not mirror-closed"
    return m


def assemble(inst, dt):
    """Assemble the linear part of the implicit balance, L I = I^n/dt + src + I0/tau.

    Row (P, d, b) holds 1/dt + 1/tau_b on the diagonal plus, for every face of P,
    v_b A_f (s_d . n_f) / V times the face intensity: the cell itself on outflow
    faces, the neighbour on interior inflow faces, the mirrored direction of the
    same cell on specular inflow wall faces; an isothermal inflow wall face puts
    its equilibrium intensity into ``src``.
    """
    nx, ny, nz = inst.n
    nc, nd, nb = nx * ny * nz, inst.s.shape[0], inst.omega.shape[0]
    dim = inst.dim
    s = inst.s.copy()
    if dim == 2:
        s[:, 2] = 0.0
    h = np.array(inst.h, dtype=float)
    if dim == 2:
        h[2] = 1.0
    mirrors = [_mirror(s, a) if any(inst.wall[f] in (1, 2) for f in (2 * a, 2 * a + 1)
                                    if f < 2 * dim) else None for a in range(3)]
    ndof = nc * nd * nb

    def lin(P, d, b):
        return (P * nd + d) * nb + b

    L = np.zeros((ndof, ndof))
    src = np.zeros(ndof)
    wall_I0 = [None if inst.wall_T[f] is None else equilibrium(inst, inst.wall_T[f])
               for f in range(6)]
    for P in range(nc):
        x, y, z = P % nx, (P // nx) % ny, P // (nx * ny)
        c = (x, y, z)
        for d in range(nd):
            for b in range(nb):
                i = lin(P, d, b)
                L[i, i] += 1.0 / dt + 1.0 / inst.tau[b]
                for f in range(2 * dim):
                    axis, plus = f // 2, f % 2
                    n_out = 1.0 if plus else -1.0
                    mu = s[d, axis] * n_out
                    coef = inst.vg[b] * mu / h[axis]  # v A mu / V, signed
                    if mu > 0:
                        L[i, i] += coef
                    elif mu < 0:
                        nbr = list(c)
                        nbr[axis] += 1 if plus else -1
                        if 0 <= nbr[axis] < inst.n[axis]:
                            Q = nbr[0] + nx * (nbr[1] + ny * nbr[2])
                            L[i, lin(Q, d, b)] += coef
                        elif inst.wall[f] == 0:
                            other = [a for a in range(3) if a != axis]
                            fi = c[other[0]] + inst.n[other[0]] * c[other[1]]
                            src[i] -= coef * wall_I0[f][fi, b]
                        elif inst.wall[f] == 3:
                            # diffuse: the outgoing flux-weighted mean of the cell
                            mu_out = s[:, axis] * n_out
                            out = mu_out > 0
                            wts = inst.w * np.where(out, mu_out, 0.0)
                            wts = wts / wts.sum()
                            for e in np.nonzero(out)[0]:
                                L[i, lin(P, e, b)] += coef * wts[e]
                        else:
                            L[i, lin(P, mirrors[axis][d], b)] += coef
    return L, src


def jacobi_sweep(inst, I_k, I_n, T_k, dt):
    """One point-Jacobi sweep of the assembled system with the equilibrium taken
    at T_k: I^{k+1} = I^k + D^{-1} (rhs - L I^k), D = diag(L)."""
    nc, nd, nb = I_k.shape
    L, src = assemble(inst, dt)
    eq = np.broadcast_to(equilibrium(inst, T_k)[:, None, :], (nc, nd, nb)).reshape(-1)
    tau_rep = np.broadcast_to(inst.tau[None, None, :], (nc, nd, nb)).reshape(-1)
    rhs = I_n.reshape(-1) / dt + src + eq / tau_rep
    Ik = I_k.reshape(-1)
    return (Ik + (rhs - L @ Ik) / np.diag(L)).reshape(nc, nd, nb)


def scattering_rate(inst, T):
    """1/tau_b at the cell temperatures T, [..., N_b]: the relaxation time
    tau_b (T0 / T)^p_b of a temperature-dependent instance, else tau_b."""
    T = np.asarray(T, dtype=complex if np.iscomplexobj(T) else float)[..., None]
    p = getattr(inst, "tau_exp", None)
    if p is None:
        return np.broadcast_to(1.0 / inst.tau, T.shape[:-1] + inst.tau.shape) + 0.0 * T
    return (T / getattr(inst, "tau_T0", 300.0)) ** p / inst.tau


def solve_backward_euler(inst, I_n, T_n, dt, t_energy=False, iters=30):
    """Solve one backward-Euler step exactly by Newton on the full system.

    I_n: [N_c, N_d, N_b]; T_n: [N_c].  Returns (I, T) at the new time level.
    The relaxation term of row (P, d, b) is (I0_b(T_P) - I) / tau_b(T_P); the
    cell's temperature equation is sum_b wgt_b(T_P) (W I0_b(T_P) - e_b) = 0 with
    e_b = sum_d w_d I and wgt_b = 1/tau_b(T) (or 1 for the plain energy sum).
    Temperature derivatives are taken by complex steps.
    """
    nx, ny, nz = inst.n
    nc, nd, nb = nx * ny * nz, inst.s.shape[0], inst.omega.shape[0]
    ndof = nc * nd * nb
    L, src = assemble(inst, dt)
    # the assembled diagonal holds the constant 1/tau_b: take it out, the
    # relaxation is added at the current temperature below
    L0 = L - np.diag(np.broadcast_to((1.0 / inst.tau)[None, None, :], (nc, nd, nb)).reshape(-1))
    W = inst.w.sum()

    def rates(T):
        return scattering_rate(inst, T)  # [nc, nb]

    def weights(T):
        return np.ones((len(T), nb)) if t_energy else rates(T)

    I = I_n.reshape(-1).copy()
    T = T_n.copy()
    rhs_n = I_n.reshape(-1) / dt + src
    for _ in range(iters):
        eq = equilibrium(inst, T)  # [nc, nb]
        phi = rates(T)
        wgt = weights(T)
        rep = lambda a: np.broadcast_to(a[:, None, :], (nc, nd, nb)).reshape(-1)  # noqa: E731
        rI = L0 @ I - rhs_n + rep(phi) * (I - rep(eq))
        Ir = I.reshape(nc, nd, nb)
        e = np.einsum("d,pdb->pb", inst.w, Ir)
        rT = (wgt * (W * eq - e)).sum(axis=1)
        # complex-step derivatives in T
        hstep = 1e-20 * T
        Tc = T + 1j * hstep
        deq = equilibrium(inst, Tc).imag / hstep[:, None]  # [nc, nb]
        dphi = rates(Tc).imag / hstep[:, None]
        dwgt = weights(Tc).imag / hstep[:, None]
        J = np.zeros((ndof + nc, ndof + nc))
        J[:ndof, :ndof] = L0 + np.diag(rep(phi))
        for P in range(nc):
            rows = np.arange(P * nd * nb, (P + 1) * nd * nb)
            IP = Ir[P]  # [nd, nb]
            J[rows, ndof + P] = (dphi[P][None, :] * (IP - eq[P][None, :])
                                 - phi[P][None, :] * deq[P][None, :]).reshape(-1)
            J[ndof + P, rows] = -np.outer(inst.w, wgt[P]).reshape(-1)
            J[ndof + P, ndof + P] = (dwgt[P] * (W * eq[P] - e[P]) + wgt[P] * W * deq[P]).sum()
        r = np.concatenate([rI, rT])
        # row scaling for conditioning
        scale = np.abs(J).max(axis=1)
        delta = np.linalg.solve(J / scale[:, None], -r / scale)
        I = I + delta[:ndof]
        T = T + delta[ndof:]
        if np.max(np.abs(delta[ndof:]) / T) < 1e-15 and \
                np.max(np.abs(delta[:ndof]) / np.abs(I)) < 1e-15:
            break
    return I.reshape(nc, nd, nb), T
