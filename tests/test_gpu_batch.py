"""Ensembles of uneven lattices (batch kernels, per-step graph and persistent schedules).

Every instance of a batch must evolve bit-for-bit as the same lattice stepped alone by lbm_step
(both run the same per-tile arithmetic), for every tile shape and schedule; a stale read across
the persistent grid barrier or a wrong tile-to-instance mapping breaks that equality.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def ensemble(orc, n=5, seed=11):
    d = synth.Draws(seed)
    cases = []
    for i in range(n):
        nx = d.choice([37, 64, 96, 130, 200])
        ny = d.choice([12, 24, 41, 64])
        form = synth.FORMS[i % 3]
        tau_v = (1.1, 2.0, 0.6)[i % 3]
        p = synth.base_params(nx=nx, ny=ny, wall_force=form, tau_v=tau_v)
        q = orc.make_params(p)
        r = max(3.0, min(nx, ny) * d.uniform(0.25, 0.4))
        rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2, 0.5)], [r], seed=seed + i)
        g = synth.gw_smooth(nx, {"rho": 0.05, "psi": -0.02, "modpsi": 0.1}[form], 0.02, seed=i)
        cases.append((dict(p, rho_l=q.rho_l, rho_v=q.rho_v), g, rho0, q))
    return cases


def plain_states(gpu, cases, steps):
    out = []
    for p, g, r, _ in cases:
        s = gpu.Sim(p, g, r)
        s.set_schedule(16 + 1)  # tile 64x8 (any tile gives the same bits)
        s.step(steps)
        out.append(s.f())
    return out


@pytest.mark.parametrize("tile,schedule", [(t, s) for t in range(5) for s in (0, 1, 2)])
def test_batch_bitwise_equals_plain(orc, gpu, tile, schedule):
    cases = ensemble(orc)
    steps = 131  # more than one captured graph chunk, odd
    ref = plain_states(gpu, cases, steps)
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": tile, "schedule": schedule})
    b.step(60)
    b.step(71)  # graph replay (64 steps) plus direct launches, odd remainder
    assert b.current_step == steps
    for i in range(len(cases)):
        assert np.array_equal(b.f(i), ref[i]), f"instance {i} differs (tile {tile}, sched {schedule})"
    obs = b.observables()
    for i, (p, g, r, q) in enumerate(cases):
        s = gpu.Sim(p, g, r)
        s.step(steps)
        o = s.observables()
        assert o["rho_min"] == obs[i]["rho_min"] and o["mass"] == obs[i]["mass"]
        assert o["n_fit"] == obs[i]["n_fit"]


def test_batch_matches_oracle(orc, gpu):
    cases = ensemble(orc, n=3, seed=5)
    steps = 200
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": 1, "schedule": 1})
    b.step(steps)
    for i, (p, g, r, q) in enumerate(cases):
        f = orc.run(q, g, orc.init_rest(q, r), steps)
        fl = orc.fluid_mask(q)
        rel = (np.abs(b.f(i) - f).max(0)[fl] / f.sum(0)[fl]).max()
        assert rel <= 1e-9, (i, rel)


def test_persistent_repeated_and_single_steps(orc, gpu):
    cases = ensemble(orc, n=4, seed=9)
    ref = plain_states(gpu, cases, 10)
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": 0, "schedule": 1})
    for n in (1, 1, 3, 3, 2):  # reused and rebuilt graphs, both parities
        b.step(n)
    for i in range(len(cases)):
        assert np.array_equal(b.f(i), ref[i])


def test_autotune_picks_a_valid_schedule(orc, gpu):
    cases = ensemble(orc, n=6, seed=3)
    best = gpu.autotune([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                        steps=20)
    print("autotune:", best)
    assert best["tile"] in (0, 1, 2, 3, 4) and best["schedule"] in (0, 1, 2) and best["ms"] > 0
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases], tune=best)
    b.step(7)
    ref = plain_states(gpu, cases, 7)
    for i in range(len(cases)):
        assert np.array_equal(b.f(i), ref[i])


def test_c3_full_size_sampled(orc, gpu):
    """The 96-lattice ensemble (128 x 64 ... 512 x 256, three forms, viscosity ratios 1, 5, 15) in
    the benchmark's launch configuration (two steps per launch, 64 x 8 output tiles): after 31
    steps, the populations of the largest and the smallest lattice and of one of each form against
    the oracle, element by element."""
    ens = synth.c3_ensemble()
    prm, gws, rhos, qs = [], [], [], []
    for e in ens:
        q = orc.make_params(e["params"])
        prm.append(dict(e["params"], rho_l=q.rho_l, rho_v=q.rho_v))
        gws.append(e["gw"])
        rhos.append(synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, e["centres"], e["radii"],
                                      seed=e["seed"]))
        qs.append(q)
    b = gpu.Batch(prm, gws, rhos, tune={"tile": 1, "schedule": 2})
    steps = 31
    b.step(steps)
    sizes = [p["nx"] * p["ny"] for p in prm]
    pick = {int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 1, 2}
    for i in sorted(pick):
        q = qs[i]
        f = orc.run(q, gws[i], orc.init_rest(q, rhos[i]), steps)
        fl = orc.fluid_mask(q)
        rel = float((np.abs(b.f(i) - f).max(0)[fl] / f.sum(0)[fl]).max())
        print(f"C3 instance {i} ({q.nx}x{q.ny}): {rel:.3e}", flush=True)
        assert rel <= 1e-9


def test_c3_viscosity_ratios_long_run(orc, gpu):
    """Phase-interpolated viscosity over a long run: the smallest lattice of the 96-lattice
    ensemble at each of the vapour/liquid viscosity ratios 5 and 15, 2,000 steps as a two-lattice
    ensemble in the benchmark's launch configuration, against the oracle element by element."""
    ens = synth.c3_ensemble()
    pick = []
    for ratio in (5.0, 15.0):
        cands = [i for i, e in enumerate(ens) if e["visc_ratio"] == ratio]
        pick.append(min(cands, key=lambda i: (ens[i]["params"]["nx"], i)))
    prm, gws, rhos, qs = [], [], [], []
    for i in pick:
        e = ens[i]
        q = orc.make_params(e["params"])
        assert q.tau_v > q.tau_l  # the viscosity varies between the phases
        prm.append(dict(e["params"], rho_l=q.rho_l, rho_v=q.rho_v))
        gws.append(e["gw"])
        rhos.append(synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, e["centres"], e["radii"],
                                      seed=e["seed"]))
        qs.append(q)
    b = gpu.Batch(prm, gws, rhos, tune={"tile": 1, "schedule": 2})
    steps = 2000
    b.step(steps)
    for k, i in enumerate(pick):
        q = qs[k]
        f = orc.run(q, gws[k], orc.init_rest(q, rhos[k]), steps)
        fl = orc.fluid_mask(q)
        rel = float((np.abs(b.f(k) - f).max(0)[fl] / f.sum(0)[fl]).max())
        print(f"C3 instance {i} ({q.nx}x{q.ny}, ratio {ens[i]['visc_ratio']:g}, "
              f"{ens[i]['form']}): {steps} steps, {rel:.3e}", flush=True)
        assert rel <= 1e-9


@pytest.mark.parametrize("schedule", [1, 2])
def test_delete_and_reallocate_without_sync(orc, gpu, schedule):
    """An ensemble dropped right after queuing steps on its own stream, with no synchronisation
    by the caller: its workspace block must not be handed to the next allocation while those
    kernels still run (the destroy call waits for the stream; the binding marks the workspace
    with record_stream), and a second run still gives the same bits."""
    import torch

    cases = ensemble(orc, n=4, seed=5)
    args = ([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases])
    tune = {"tile": 1, "schedule": schedule}
    b = gpu.Batch(*args, tune=tune)
    b.step(200)
    ref = [b.f(i) for i in range(len(cases))]
    del b
    for _ in range(3):
        b = gpu.Batch(*args, tune=tune)
        nbytes = b.ws.numel()
        b.step(200)
        del b  # no synchronisation before the block goes back to torch's allocator
        x = torch.full((nbytes // 8,), 7.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        assert bool((x == 7.0).all()), "a freed workspace block was written after reuse"
        del x
    b = gpu.Batch(*args, tune=tune)
    b.step(200)
    for i in range(len(cases)):
        assert np.array_equal(b.f(i), ref[i])


@pytest.mark.parametrize("tile", [1, 2])
def test_persistent_full_size_bitwise_equals_graph(orc, gpu, tile):
    """The 96-lattice ensemble with the persistent schedule (one launch of 40 steps: 20 two-step
    passes, every barrier after the first through the per-XCD leaders) against graph-replayed
    two-step launches of the same tiles, every instance bit for bit; at full size every XCD runs
    dozens of workgroups, each taking many tiles per pass from its XCD's ticket counter."""
    ens = synth.c3_ensemble()
    prm, gws, rhos = [], [], []
    for e in ens:
        q = orc.make_params(e["params"])
        prm.append(dict(e["params"], rho_l=q.rho_l, rho_v=q.rho_v))
        gws.append(e["gw"])
        rhos.append(synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, e["centres"], e["radii"],
                                      seed=e["seed"]))
    out = []
    for schedule in (2, 1):
        b = gpu.Batch(prm, gws, rhos, tune={"tile": tile, "schedule": schedule})
        b.step(40)
        out.append([b.f(i) for i in range(len(prm))])
        del b
    for i in range(len(prm)):
        assert np.array_equal(out[0][i], out[1][i]), f"instance {i} differs (tile {tile})"


def test_persistent_barrier_timeout_aborts_cleanly(orc, gpu, monkeypatch):
    """A persistent run whose barrier waits may not poll at all (LBM_PERSISTENT_SPIN_LIMIT=0, read
    when the ensemble is created): every workgroup leaves through the abort flag instead of
    waiting, the next observables call reports the time-out, and a new ensemble created without
    the setting runs normally, bit for bit as the plain runs."""
    cases = ensemble(orc, n=4, seed=5)
    args = ([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases])
    tune = {"tile": 1, "schedule": 1}
    monkeypatch.setenv("LBM_PERSISTENT_SPIN_LIMIT", "0")
    b = gpu.Batch(*args, tune=tune)
    monkeypatch.delenv("LBM_PERSISTENT_SPIN_LIMIT")
    b.step(40)
    with pytest.raises(gpu.LBMError) as e:
        b.observables()
    assert "timed out" in str(e.value)
    del b
    ref = plain_states(gpu, cases, 40)
    b = gpu.Batch(*args, tune=tune)
    b.step(40)
    for i in range(len(cases)):
        assert np.array_equal(b.f(i), ref[i])



@pytest.mark.parametrize("tile", [4, 0])
def test_persistent_many_passes_small_tiles(orc, gpu, tile):
    """Small tiles of small lattices, whose data a compute unit's L1 keeps from one pass to the
    next: 1,000 steps (500 passes, each barrier after the first through the per-XCD leaders) of
    the persistent schedule against graph-replayed two-step launches, bit for bit. A barrier
    whose waiting workgroups do not invalidate their L1 reads stale lines here."""
    cases = ensemble(orc)
    args = ([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases])
    out = []
    for schedule in (2, 1):
        b = gpu.Batch(*args, tune={"tile": tile, "schedule": schedule})
        b.step(1000)
        out.append([b.f(i) for i in range(len(cases))])
        del b
    for i in range(len(cases)):
        assert np.array_equal(out[0][i], out[1][i]), f"instance {i} differs (tile {tile})"
