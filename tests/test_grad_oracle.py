"""Pins of the gradient oracle (PyTorch CPU float64 + autograd) against the C oracle: the forward
states agree to round-off and the gradient agrees with central finite differences of the C
oracle's objective (no GPU)."""
import numpy as np
import pytest

import synth


def case(orc, form, nx=40, ny=20, tau_v=2.0, ghost=1):
    p = synth.base_params(nx=nx, ny=ny, wall_force=form, tau_v=tau_v, ghost=ghost)
    q = orc.make_params(p)
    # without the mirrored ghost rows a droplet touching the wall is unstable (the solid acts as
    # psi = 0 to the cohesive force), so that case keeps the droplet off the wall
    c, R = ((nx / 2, 0.5), 8.0) if ghost else ((nx / 2, ny / 2), 5.0)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [c], [R], seed=3)
    gw = synth.gw_smooth(nx, {"rho": 0.05, "psi": -0.02, "modpsi": 0.1}[form], 0.03, seed=2)
    gw[1] = np.linspace(-0.02, 0.02, nx)
    return q, gw, orc.init_rest(q, rho0)


@pytest.mark.parametrize("form,ghost", [("rho", 1), ("psi", 1), ("modpsi", 1), ("modpsi", 0)])
def test_gradient_oracle_forward_and_fd(orc, form, ghost):
    from oracle import grad_oracle as G
    q, gw, f0 = case(orc, form, ghost=ghost)
    n = 80
    fc = orc.run(q, gw, f0.copy(), n)
    ft = G.forward_state(f0, gw, q, n)
    fl = orc.fluid_mask(q)
    assert (np.abs(fc - ft).max(0)[fl] / fc.sum(0)[fl]).max() <= 1e-12
    L, g = G.loss_and_grad(f0, gw, q, n)
    assert abs(L - orc.loss(q, fc.sum(0))) <= 1e-12 * abs(L)
    scale = np.abs(g).max()
    h = 1e-5
    for w, x in [(0, 3), (0, 20), (0, 27), (1, 11)]:
        vals = []
        for sgn in (1, -1):
            gg = gw.copy(); gg[w, x] += sgn * h
            vals.append(orc.loss(q, orc.run(q, gg, f0.copy(), n).sum(0)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[w, x] - fd) <= 1e-6 * scale, (w, x, g[w, x], fd)


@pytest.mark.parametrize("form,gw_mean", [("modpsi", 0.3), ("rho", 0.15), ("psi", -1.0)])
def test_gradient_oracle_piecewise_eos(orc, form, gw_mean):
    """The same pins with the paper's Eq. (15) EOS at 500/1 (sigma = 0.084, viscosity ratio
    nu_V/nu_L = 5): forward states against the C oracle to round-off, the objective, and the
    gradient against central differences of the C oracle's objective."""
    from oracle import grad_oracle as G
    nx, ny, n = 40, 20, 80
    p = dict(nx=nx, ny=ny, walls=1, ghost=1, eos="piecewise", th_v=0.64 / 3, th_m=-0.04 / 3,
             th_l=1 / 3, rho_v=1.0, rho_l=500.0, G=-1.0, sigma=0.084, tau_l=1.1, tau_v=2.0,
             wall_force=form, **synth.RATES)
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2, 0.5)], [8.0], width=4.0,
                             seed=3)
    gw = synth.gw_smooth(nx, gw_mean, abs(gw_mean) * 0.3, seed=2)
    gw[1] = np.linspace(-0.02, 0.02, nx)
    f0 = orc.init_rest(q, rho0)
    fc = orc.run(q, gw, f0.copy(), n)
    ft = G.forward_state(f0, gw, q, n)
    fl = orc.fluid_mask(q)
    assert (np.abs(fc - ft).max(0)[fl] / fc.sum(0)[fl]).max() <= 1e-12
    L, g = G.loss_and_grad(f0, gw, q, n)
    assert abs(L - orc.loss(q, fc.sum(0))) <= 1e-12 * abs(L)
    scale = np.abs(g).max()
    h = 1e-5
    for w, x in [(0, 3), (0, 20), (0, 27), (1, 11)]:
        vals = []
        for sgn in (1, -1):
            gg = gw.copy(); gg[w, x] += sgn * h
            vals.append(orc.loss(q, orc.run(q, gg, f0.copy(), n).sum(0)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[w, x] - fd) <= 1e-6 * scale, (w, x, g[w, x], fd)


def test_streaming_is_a_permutation_inverted_by_its_transpose():
    """Streaming with halfway bounce-back moves every post-collision population to exactly one
    place: the streamed field holds the same values, and the transposed map (the vector-Jacobian
    product, which the adjoint's transposed streaming computes) applied to it gives the input
    back bit for bit."""
    import torch
    from oracle import grad_oracle as G
    torch.manual_seed(0)
    for ny_f, nx in ((6, 9), (2, 5), (11, 3)):
        fs = torch.rand((9, ny_f, nx), dtype=torch.float64)
        out = G.stream(fs)
        assert torch.equal(torch.sort(out.flatten()).values, torch.sort(fs.flatten()).values)
        _, vjp = torch.func.vjp(G.stream, fs)
        (back,) = vjp(out)
        assert torch.equal(back, fs)
