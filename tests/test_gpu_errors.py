"""Error paths of the device entry points.

kpm_debug_inject_failure makes the n-th checked HIP operation of the library
fail (an allocation or enqueue is skipped, a synchronising call or a launch
check has its status replaced).  For each entry point below the failure is
moved over every checked operation of one call in turn (n = 1, 2, ... until
the call no longer reaches the n-th), with both injected kinds, and each time

  * the call returns KPM_E_NOMEM (out of memory) or KPM_E_DEVICE (launch
    failure) with a message naming the failed operation,
  * every device buffer the call allocated is released again
    (kpm_debug_live_allocations back to its value before the call),
  * the library keeps working: the run after the sweep gives the clean run's
    result bit for bit.

Two real failures complete the set: a DOS plan too large for HBM (hipMalloc
itself fails) and a Gamma batch that cannot hold one vector (the size check
before any allocation).
"""
import numpy as np
import pytest

import workload as wl

pytestmark = pytest.mark.gpu

MAX_STEPS = 4000   # more checked operations than any call below makes


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05194_amd import kpm
    return kpm


def _sweep(K, name, call, kinds=(0, 1)):
    """Inject a failure at every checked operation of call(); return the clean result
    of the first call that completes and the number of checked operations seen."""
    import torch
    expect = {0: K.KPM_E_NOMEM, 1: K.KPM_E_DEVICE}
    text = {0: "out of memory", 1: "launch failure"}   # hipGetErrorString of the injected errors
    results = {}
    for kind in kinds:
        n = 1
        while True:
            assert n < MAX_STEPS, f"{name}: no end to the checked operations"
            live = K.debug_live_allocations()
            K.debug_inject_failure(n, kind)
            err, out = None, None
            try:
                out = call()
            except K.KPMError as e:
                err = e
            fired = K.debug_inject_failure(0, 0)
            torch.cuda.synchronize()
            assert K.debug_live_allocations() == live, f"{name}: buffers left after failure {n} (kind {kind})"
            if not fired:
                assert err is None, f"{name}: failed without an injected failure: {err}"
                results[kind] = (out, n - 1)
                break
            assert err is not None, f"{name}: injected failure {n} (kind {kind}) was not reported"
            assert err.code == expect[kind], f"{name}: failure {n} kind {kind} gave {err.code}: {err}"
            assert text[kind] in str(err), f"{name}: failure {n}: {err}"
            n += 1
        print(f"{name}: kind {kind}: {results[kind][1]} checked operations, every failure reported", flush=True)
    return results


def _dos_case():
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=40, L2=36, t=-2.7, anderson_w=0.8, vacancy_p=0.03, disorder_seed=5)
    par = wl.DosParams(num_moments=64, num_random=3, vector_seed=21, precision=wl.FP32)
    return lat, par


def test_dos_one_shot_every_failure(K):
    lat, par = _dos_case()
    ref, _ = K.moments_dos([lat], par)
    res = _sweep(K, "kpm_moments_dos", lambda: K.moments_dos([lat], par)[0])
    for kind, (mu, n) in res.items():
        assert n >= 20
        assert np.array_equal(mu, ref)


def test_plan_with_graph_every_failure(K):
    import torch
    lat, par = _dos_case()
    ref = K.moments_dos([lat], par)[1]

    def call():
        plan = K.Plan([lat], par, use_graph=True)
        try:
            mean = torch.zeros((1, par.num_moments), dtype=torch.float64, device="cuda")
            plan.run(None, mean)
            plan.run(None, mean)   # second run replays the captured graph
            torch.cuda.synchronize()
            return mean.cpu().numpy()
        finally:
            plan.close()

    res = _sweep(K, "kpm_plan_create/run (graph)", call)
    for kind, (mean, n) in res.items():
        assert np.array_equal(mean, ref)


def test_noalloc_every_failure(K):
    lat, par = _dos_case()
    ref = K.moments_dos([lat], par)[0]
    res = _sweep(K, "kpm_moments_dos_noalloc", lambda: K.moments_dos_noalloc([lat], par)[0])
    for kind, (mu, n) in res.items():
        assert np.array_equal(mu, ref)


@pytest.mark.parametrize("steps", ["1", "4"], ids=["single-steps", "sweeps"])
def test_gamma_every_failure(K, monkeypatch, steps):
    """Split-BF16 Gamma over two batches of vectors (max_batch = 1), and the FP64 GEMM,
    with the chains as single steps and as four-step sweeps."""
    monkeypatch.setenv("KPM_CHAIN_STEPS", steps)
    lat = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=8, L2=6, t=-2.7, rashba=0.4, anderson_w=0.6, disorder_seed=3,
                     e_min=-9.0, e_max=9.0)
    M = 24
    for mode in (wl.GAMMA_SPLIT_BF16, wl.GAMMA_FP64):
        par = wl.CondParams(num_moments=M, num_random=2, vector_seed=9, alpha=0, beta=1, gamma_mode=mode)
        ref = K.moments_cond(lat, par, precision=wl.FP32, max_batch=1)
        res = _sweep(K, f"kpm_moments_cond (mode {mode}, KPM_CHAIN_STEPS={steps})",
                     lambda: K.moments_cond(lat, par, precision=wl.FP32, max_batch=1))
        for kind, (G, n) in res.items():
            # two batches, each with at least one checked launch per chain step or sweep
            assert n >= 2 * 2 * (M // int(steps))
            assert np.array_equal(G, ref)


def test_gamma1_and_reconstruction_every_failure(K):
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=12, L2=10, t=-2.7, anderson_w=1.0, disorder_seed=2)
    par = wl.CondParams(num_moments=32, num_random=2, vector_seed=4, alpha=0, beta=0, gamma_mode=wl.GAMMA_FP64)
    g1 = K.moments_gamma1(lat, par, precision=wl.FP64)
    res = _sweep(K, "kpm_moments_gamma1", lambda: K.moments_gamma1(lat, par, precision=wl.FP64))
    for kind, (g, n) in res.items():
        assert np.array_equal(g, g1)
    mu = K.moments_dos([lat], wl.DosParams(num_moments=32, num_random=2, vector_seed=4, precision=wl.FP64))[1][0]
    E = np.linspace(-7.0, 7.0, 50)
    rho = K.reconstruct_jackson(mu, E, lat.e_min, lat.e_max)
    res = _sweep(K, "kpm_reconstruct_jackson", lambda: K.reconstruct_jackson(mu, E, lat.e_min, lat.e_max))
    for kind, (r, n) in res.items():
        assert np.array_equal(r, rho)
    G = K.moments_cond(lat, par, precision=wl.FP64)
    sig = K.reconstruct_sigma(G, E, lat.e_min, lat.e_max, 1.0)
    res = _sweep(K, "kpm_reconstruct_sigma", lambda: K.reconstruct_sigma(G, E, lat.e_min, lat.e_max, 1.0))
    for kind, (s, n) in res.items():
        assert np.array_equal(s, sig)
    sb = K.reconstruct_sigma_bastin(G, E[:8], lat.e_min, lat.e_max, 0.05, 1.0)
    res = _sweep(K, "kpm_reconstruct_sigma_bastin",
                 lambda: K.reconstruct_sigma_bastin(G, E[:8], lat.e_min, lat.e_max, 0.05, 1.0))
    for kind, (s, n) in res.items():
        assert np.array_equal(s, sb)


def test_mlp_every_failure(K):
    """Create, fit the standardisation, one training step and a forward pass: a failure
    anywhere leaves no buffer behind once the network is destroyed, and a network that
    saw a failed call still trains (its workspace is rebuilt)."""
    import torch
    g = np.random.default_rng(3)
    X = torch.tensor(g.normal(size=(48, 32)) * 0.1, dtype=torch.float32, device="cuda")
    T = torch.tensor(g.normal(size=(48, 16)) * 0.01, dtype=torch.float32, device="cuda")
    w = torch.ones(16, dtype=torch.float32, device="cuda")

    def call():
        net = K.MLP(32, 64, 16, seed=5)
        try:
            net.fit_scaling(X, T)
            loss = torch.zeros(1, dtype=torch.float64, device="cuda")
            net.train_step(X, T, w, 1e-3, loss_out=loss)
            y = net.forward(X)
            torch.cuda.synchronize()
            return y.cpu().numpy(), loss.cpu().numpy()
        finally:
            net.close()

    ref = call()
    res = _sweep(K, "kpm_mlp_*", call)
    for kind, ((y, loss), n) in res.items():
        assert np.array_equal(y, ref[0]) and np.array_equal(loss, ref[1])
    # A network whose workspace allocation failed rebuilds it on the next call.
    net = K.MLP(32, 64, 16, seed=5)
    try:
        net.fit_scaling(X, T)
        K.debug_inject_failure(1, 0)
        with pytest.raises(K.KPMError) as e:
            net.forward(X)
        assert K.debug_inject_failure(0, 0) == 1 and e.value.code == K.KPM_E_NOMEM
        y = net.forward(X)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(y.cpu().numpy()))
    finally:
        net.close()


def test_time_evolve_every_failure(K):
    lat = wl.Lattice(kind=wl.HONEYCOMB, L1=10, L2=8, t=-2.7, anderson_w=0.5, disorder_seed=6)
    g = np.random.default_rng(1)
    psi0 = g.normal(size=(2, lat.n_orbitals)) + 1j * g.normal(size=(2, lat.n_orbitals))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    ref = K.time_evolve(lat, psi0, 0.5, 40, 3, precision=wl.FP64)
    res = _sweep(K, "kpm_time_evolve", lambda: K.time_evolve(lat, psi0, 0.5, 40, 3, precision=wl.FP64))
    for kind, ((psi, obs), n) in res.items():
        assert np.array_equal(psi, ref[0]) and np.array_equal(obs, ref[1])


def test_real_out_of_memory(K):
    """Allocations the device cannot hold fail as KPM_E_NOMEM, with nothing left
    allocated and the library usable afterwards."""
    import torch
    live = K.debug_live_allocations()
    # 32768 x 32768 honeycomb cells, 16 FP64 vectors: 550 GB per Chebyshev vector.
    big = wl.Lattice(kind=wl.HONEYCOMB, L1=32768, L2=32768, t=-2.7)
    par = wl.DosParams(num_moments=16, num_random=16, vector_seed=1, precision=wl.FP64)
    print("real OOM: DOS plan of 32768 x 32768 honeycomb cells, R = 16, FP64", flush=True)
    with pytest.raises(K.KPMError) as e:
        K.Plan([big], par)
    assert e.value.code == K.KPM_E_NOMEM, str(e.value)
    assert "device allocation of 549755813888 bytes failed" in str(e.value), str(e.value)
    assert K.debug_live_allocations() == live
    # Gamma: two [M][N][R] blocks of one vector exceed the device: refused before allocating.
    spin = wl.Lattice(kind=wl.HONEYCOMB_SPIN, L1=4096, L2=4096, t=-2.7, rashba=0.3)
    cp = wl.CondParams(num_moments=4096, num_random=1, vector_seed=1, alpha=0, beta=1)
    print("real OOM: Gamma blocks of 4096 x 4096 spinful cells, M = 4096", flush=True)
    with pytest.raises(K.KPMError) as e:
        K.moments_cond(spin, cp)
    assert e.value.code == K.KPM_E_NOMEM and "not enough device memory" in str(e.value), str(e.value)
    assert K.debug_live_allocations() == live
    lat, dpar = _dos_case()
    mu, _ = K.moments_dos([lat], dpar)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(mu))


def test_kpm_log_plan_summary(K, capfd, monkeypatch):
    """KPM_LOG=1 makes plan creation print one summary line of the chosen plan to
    stderr, with the launch shape kpm_plan_info reports."""
    lat, par = _dos_case()
    monkeypatch.setenv("KPM_LOG", "1")
    plan = K.Plan([lat], par, use_graph=False)
    info = plan.info()
    plan.close()
    K.moments_dos([lat], par)
    K.moments_dos_noalloc([lat], par)
    monkeypatch.setenv("KPM_LOG", "0")
    K.moments_dos([lat], par)
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("[kpm] plan:")]
    assert len(lines) == 3, err
    n_orb = 2 * lat.L1 * lat.L2
    for l in lines:
        print(l)
        assert f"{n_orb} orbitals" in l and "R=3 (padded 4)" in l and "M=64" in l and "fp32" in l, l
        assert f"kernel {info['kernel']} " in l and f"block {info['block']}," in l, l
        assert (f"tile {info['tile_cells_x']} cells x {info['rows']} rows x {info['tile_chunks']} chunks, "
                f"grid {info['grid']}, {info['n_tiles']} tiles") in l, l
    assert "(scratch array)" in lines[2] and "(scratch array)" not in lines[0]
