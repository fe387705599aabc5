"""Reference gradients of the wetting objective with respect to G_w (TEST INFRASTRUCTURE).

A second, vectorised statement of the same time step in plain PyTorch CPU float64 operations,
differentiated by torch.autograd. Walls at rows 0 and ny-1 (the objective needs them). Same
order of operations as the paper: density and pseudopotential, cohesive force Eq. (7),
adhesive force Eq. (10)/(11)/(14), velocity Eq. (6), moments, equilibria Eq. (3), forcing
Eq. (9), relaxation Eq. (4), f* = M^-1 m*, streaming Eq. (5) with halfway bounce-back.
It is checked against the C oracle (forward) and against central differences (gradient).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

EX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
EY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
OPP = (0, 3, 4, 1, 2, 7, 8, 5, 6)
W = (0.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12)
# Lallemand-Luo moment basis: rows (rho, e, epsilon, jx, qx, jy, qy, pxx, pxy)
M = torch.tensor([[1, 1, 1, 1, 1, 1, 1, 1, 1],
                  [-4, -1, -1, -1, -1, 2, 2, 2, 2],
                  [4, -2, -2, -2, -2, 1, 1, 1, 1],
                  [0, 1, 0, -1, 0, 1, -1, -1, 1],
                  [0, -2, 0, 2, 0, 1, -1, -1, 1],
                  [0, 0, 1, 0, -1, 1, 1, -1, -1],
                  [0, 0, -2, 0, 2, 1, 1, -1, -1],
                  [0, 1, -1, 1, -1, 0, 0, 0, 0],
                  [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=torch.float64)
MINV = torch.linalg.inv(M)


def p_eos(rho, q):
    if q.eos == 0:
        eta = q.b * rho / 4
        return rho * q.R * q.T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - q.a * rho ** 2
    p1 = q.rho1 * q.th_v
    p2 = p1 + (q.rho2 - q.rho1) * q.th_m
    return torch.where(rho <= q.rho1, rho * q.th_v,
                       torch.where(rho <= q.rho2, p1 + (rho - q.rho1) * q.th_m,
                                   p2 + (rho - q.rho2) * q.th_l))


def step(F, gw, q):
    """One step on the fluid rows. F: (9, ny-2, nx) pre-collision populations; gw: (2, nx)."""
    nyf = F.shape[1]
    rho = F.sum(0)
    psi = torch.sqrt(2 * (p_eos(rho, q) - rho / 3) / q.G)
    if q.ghost:
        P = torch.cat([psi[:1], psi, psi[-1:]], 0)      # mirrored solid rows
    else:
        z = torch.zeros_like(psi[:1])
        P = torch.cat([z, psi, z], 0)

    def at(dx, dy):  # psi(x + dx, y + dy) on the fluid rows
        return torch.roll(P, shifts=-dx, dims=1)[1 + dy:1 + dy + nyf]

    sx = sum(W[a] * EX[a] * at(EX[a], EY[a]) for a in range(1, 9))
    sy = sum(W[a] * EY[a] * at(EX[a], EY[a]) for a in range(1, 9))
    Fmx, Fmy = -q.G * psi * sx, -q.G * psi * sy

    pre = rho if q.wall_force == 0 else (psi if q.wall_force == 1 else psi * psi)
    zero_row = torch.zeros_like(gw[0])
    ax_b, ay_b, ax_t, ay_t = zero_row, zero_row, zero_row, zero_row
    for a in range(1, 9):
        om = W[a] / 3
        if EY[a] == -1:   # solid node below the first fluid row
            g = torch.roll(gw[0], shifts=-EX[a])
            ax_b = ax_b + om * g * EX[a]
            ay_b = ay_b + om * g * EY[a]
        if EY[a] == 1:    # solid node above the last fluid row
            g = torch.roll(gw[1], shifts=-EX[a])
            ax_t = ax_t + om * g * EX[a]
            ay_t = ay_t + om * g * EY[a]
    mid = torch.zeros((nyf - 2, gw.shape[1]), dtype=F.dtype)  # walls need ny >= 4: nyf >= 2
    Ax = torch.cat([ax_b[None], mid, ax_t[None]], 0)
    Ay = torch.cat([ay_b[None], mid, ay_t[None]], 0)
    Fx, Fy = Fmx - pre * Ax, Fmy - pre * Ay

    jx = sum(EX[a] * F[a] for a in range(9))
    jy = sum(EY[a] * F[a] for a in range(9))
    vx, vy = (jx + Fx / 2) / rho, (jy + Fy / 2) / rho
    v2 = vx * vx + vy * vy
    m = torch.einsum("ka,ayx->kyx", M, F)
    meq = torch.stack([rho, rho * (-2 + 3 * v2), rho * (1 - 3 * v2), rho * vx, -rho * vx,
                       rho * vy, -rho * vy, rho * (vx * vx - vy * vy), rho * vx * vy])
    nu_l, nu_v = (q.tau_l - 0.5) / 3, (q.tau_v - 0.5) / 3
    phi = torch.clamp((rho - q.rho_v) / (q.rho_l - q.rho_v), 0.0, 1.0)
    snu = 1 / (3 * (nu_v + phi * (nu_l - nu_v)) + 0.5)
    one = torch.ones_like(rho)
    s = torch.stack([q.s_rho * one, q.s_e * one, q.s_zeta * one, q.s_j * one, q.s_q * one,
                     q.s_j * one, q.s_q * one, snu, snu])
    Fm2 = Fmx * Fmx + Fmy * Fmy
    vF = vx * Fx + vy * Fy
    tau_e, tau_z = 1 / q.s_e, 1 / q.s_zeta
    S = torch.stack([0 * rho, 6 * vF + 12 * q.sigma * Fm2 / (psi * psi * (tau_e - 0.5)),
                     -6 * vF - 12 * q.sigma * Fm2 / (psi * psi * (tau_z - 0.5)),
                     Fx, -Fx, Fy, -Fy, 2 * (vx * Fx - vy * Fy), vx * Fy + vy * Fx])
    ms = m - s * (m - meq) + (1 - s / 2) * S
    fs = torch.einsum("ak,kyx->ayx", MINV, ms)
    return stream(fs)


def stream(fs):
    """Eq. (5) with halfway bounce-back on the fluid rows: f_a(x) = f*_a(x - e_a), or f*_opp(a)(x)
    when x - e_a lies in a solid row; x periodic."""
    out = []
    for a in range(9):
        src = torch.roll(fs[a], shifts=EX[a], dims=1)
        if EY[a] == 0:
            out.append(src)
        elif EY[a] == 1:   # arriving from below; the first row is fed by the bottom wall
            out.append(torch.cat([fs[OPP[a]][:1], src[:-1]], 0))
        else:              # arriving from above; the last row is fed by the top wall
            out.append(torch.cat([src[1:], fs[OPP[a]][-1:]], 0))
    return torch.stack(out)


def objective(F, q, w_centroid=1.0, w_wet=1.0):
    rho = F.sum(0)
    phi = (rho - q.rho_v) / (q.rho_l - q.rho_v)
    y = torch.arange(1, F.shape[1] + 1, dtype=F.dtype)[:, None] - 0.5
    yc = (phi * y).sum() / phi.sum()
    lw = phi[0].sum()
    return w_centroid * yc + w_wet * lw


def run(F0, gw, q, nsteps, chunk=50):
    """nsteps steps; chunks are recomputed in the backward pass to bound memory."""
    F = F0

    def many(F, gw, n):
        for _ in range(n):
            F = step(F, gw, q)
        return F

    done = 0
    while done < nsteps:
        n = min(chunk, nsteps - done)
        if gw.requires_grad:
            F = checkpoint(many, F, gw, n, use_reentrant=False)
        else:
            F = many(F, gw, n)
        done += n
    return F


def loss_and_grad(f0, gw, q, nsteps, w_centroid=1.0, w_wet=1.0, chunk=50):
    """Objective after nsteps from f0 (9, ny, nx, numpy, walls) and dL/dG_w (2, nx)."""
    torch.set_num_threads(max(1, torch.get_num_threads()))
    F0 = torch.tensor(f0[:, 1:-1, :], dtype=torch.float64)
    g = torch.tensor(gw, dtype=torch.float64, requires_grad=True)
    L = objective(run(F0, g, q, nsteps, chunk), q, w_centroid, w_wet)
    L.backward()
    return float(L), g.grad.numpy().copy()


def forward_state(f0, gw, q, nsteps):
    """Populations after nsteps, (9, ny, nx) with zero solid rows."""
    import numpy as np
    F0 = torch.tensor(f0[:, 1:-1, :], dtype=torch.float64)
    with torch.no_grad():
        F = run(F0, torch.tensor(gw, dtype=torch.float64), q, nsteps)
    out = np.zeros_like(f0)
    out[:, 1:-1, :] = F.numpy()
    return out
