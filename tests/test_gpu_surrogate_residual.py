"""GPU tests of the residual form of the learned dipole field
(sp_ddi_init_residual) against the FP64 oracle: the backbone (exact near
blocks plus far block dipoles), the full field with a given network
(bf16 contract on the network's correction), and what training gives: the
field error against the FP64 direct sum with the trained network and
without it (the backbone alone) on held-out textures."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu

HAM4 = si.WORKLOADS["film128x4_dipolar"].hamiltonian
C_DD = 1.00000000055e-7 * 9.2740100783e-24 ** 2 / 1e-30 / 1.602176634e-22
MU = HAM4.mu[0]
SCALE = C_DD * MU * MU
BLOCK, REACH = 4, 2
CHANNELS = [12, 32, 32, 32, 12]
# the residual form's documented scales (lattice constant 1 Angstrom)
IN_S = np.array([1 / 64] * 3 + [1 / 16] * 9)
OUT_S = np.array([4e-3] * 3 + [1e-3] * 9)


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _film(L=64):
    return si.simple_cubic(L, L, 4, periodic=(0, 0, 0))


def _engine(geo, seed=1):
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, "f32")
    e.set_geometry(geo)
    e.set_hamiltonian(dataclasses.replace(HAM4, ddi=True))
    e.ddi_init_residual(CHANNELS, seed=seed, block=BLOCK, reach=REACH)
    return e


def _texture(geo, k):
    W, H, _ = geo.n_cells
    r = np.random.default_rng(5000 + k)
    kind = k % 3
    if kind == 0:
        return si.uniform_sphere(geo.n_sites, 7000 + k)
    if kind == 1:
        return si.domain_walls(geo, n_walls=int(r.integers(1, 4)), seed=7000 + k, bloch=bool(r.integers(2)))
    return si.skyrmion_ansatz(geo, radius=float(r.uniform(4, 0.3 * W)),
                              center=(float(r.uniform(0.25, 0.75) * W), float(r.uniform(0.25, 0.75) * H)),
                              helicity=float(r.uniform(0, 6.283)), width=float(r.uniform(1.5, 4.0)), noise_rad=0.05,
                              seed=7000 + k)


def _f32(n):
    return np.asarray(n, dtype=np.float32).astype(np.float64)


def _oracle_system(ora, geo):
    return ora.System(geo, si.Hamiltonian(mu=HAM4.mu, B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), ddi=True))


def test_residual_backbone_matches_oracle(ora):
    import torch

    announce("residual backbone 64x64x4")
    geo = _film()
    e = _engine(geo)
    s = _oracle_system(ora, geo)
    n = np.stack([_f32(_texture(geo, k)) for k in range(3)])
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    ft = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_backbone_dev(3, nt, ft)
    e.synchronize()
    got = ft.cpu().numpy().astype(np.float64)
    for b in range(3):
        ref = s.ddr_backbone(n[b], BLOCK, REACH) * SCALE
        assert rel_err(got[b], ref) <= 1e-5, b
    e.close()


def _seeded_params(ora, seed, scale=0.15):
    nparam = sum(9 * a * b + b for a, b in zip(CHANNELS[:-1], CHANNELS[1:]))
    return ora.bf16(np.random.default_rng(seed).standard_normal(nparam) * scale)


def _layers(p):
    ws, bs, q = [], [], 0
    for a, b in zip(CHANNELS[:-1], CHANNELS[1:]):
        ws.append(p[q:q + 9 * a * b].reshape(3, 3, a, b))
        q += 9 * a * b
        bs.append(p[q:q + b])
        q += b
    return ws, bs


def test_residual_forward_matches_oracle(ora):
    """Field = scale (backbone + per-block correction of the network on the
    scaled block moments).  The correction is compared on its own scale: the
    network input is rounded to bf16 on both sides from moments summed in
    FP32 (GPU) or FP64 (oracle), so an input next to a rounding boundary may
    round one bf16 ulp apart; such flips and the bf16 activations bound the
    correction's difference by a few bf16 ulps (2^-7 normwise)."""
    import torch

    announce("residual forward 64x64x4")
    geo = _film()
    e = _engine(geo)
    p = _seeded_params(ora, 77)
    e.ddi_set_params(p)
    s = _oracle_system(ora, geo)
    n = np.stack([_f32(_texture(geo, k)) for k in range(3, 5)])
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    full, back = torch.zeros_like(nt), torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_forward_dev(2, nt, full)
    e.ddi_backbone_dev(2, nt, back)
    e.synchronize()
    corr_gpu = (full - back).cpu().numpy().astype(np.float64)
    ws, bs = _layers(p)
    net = ora.SurrogateNet(ws, bs)
    for b in range(2):
        x = ora.bf16(s.ddr_moments(n[b], BLOCK) * IN_S)[None]
        z = net.forward(x)[0]
        corr = s.ddr_expand(z * OUT_S, BLOCK) * SCALE
        assert rel_err(corr_gpu[b], corr) <= 2.0 ** -7, b
    e.close()


def test_trained_network_gains_over_the_backbone_against_the_fp64_oracle(ora):
    """Train on 240 textures of a 64 x 64 x 4 film (labels from the GPU
    direct sum), then on 20 held-out textures compare, at 256 sampled sites
    each, the field with the trained network and the backbone alone with the
    FP64 oracle's direct sum.  The network must cut the mean error by at
    least a third (the gain); both errors are printed next to the 1e-3
    residual-check tolerance."""
    import torch

    announce("residual training gain 64x64x4")
    geo = _film()
    e = _engine(geo, seed=2)
    ntrain, ntest = 240, 20
    tex = np.stack([_f32(_texture(geo, k)) for k in range(ntrain + ntest)])
    nt = torch.tensor(tex, dtype=torch.float32, device="cuda").contiguous()
    lab = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_label_dev(ntrain + ntest, nt, lab)
    losses = e.ddi_train_dev(ntrain, nt[:ntrain].contiguous(), lab[:ntrain].contiguous(), epochs=40, batch=8,
                             lr=2e-3, seed=0)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    test = nt[ntrain:].contiguous()
    with_net, without = torch.zeros_like(test), torch.zeros_like(test)
    e.ddi_forward_dev(ntest, test, with_net)
    e.ddi_backbone_dev(ntest, test, without)
    e.synchronize()
    wn, wo = with_net.cpu().numpy().astype(np.float64), without.cpu().numpy().astype(np.float64)
    s = _oracle_system(ora, geo)
    rng = np.random.default_rng(3)
    err_w, err_o = [], []
    for b in range(ntest):
        sites = np.sort(rng.choice(geo.n_sites, 256, replace=False))
        exact = s.dipole_gradient_sites(tex[ntrain + b], sites)
        nrm = np.linalg.norm(exact)
        err_w.append(np.linalg.norm(wn[b][:, sites] - exact) / nrm)
        err_o.append(np.linalg.norm(wo[b][:, sites] - exact) / nrm)
    err_w, err_o = np.array(err_w), np.array(err_o)
    print(f"[residual] held-out field error vs FP64 oracle: with network mean {err_w.mean():.2e} "
          f"max {err_w.max():.2e}; backbone alone mean {err_o.mean():.2e} max {err_o.max():.2e}; "
          f"below 1e-3: {int((err_w < 1e-3).sum())}/{ntest} with, {int((err_o < 1e-3).sum())}/{ntest} without",
          flush=True)
    assert err_w.mean() < (2.0 / 3.0) * err_o.mean()
    e.close()


def test_full_size_film_error_against_the_fp64_oracle(ora):
    """The 128 x 128 x 4 film: train on 600 textures (a third relaxed
    skyrmion/bubble textures), then the field error against the FP64 oracle
    at 256 sampled sites of each of 24 held-out textures, with the network
    and with the backbone alone."""
    import torch

    import bench
    import paper_1901_11350_amd as pk

    announce("residual full-size film 128x128x4")
    w = si.WORKLOADS["film128x4_dipolar"]
    geo = w.geometry
    e = _engine(geo, seed=4)
    f = pk.Engine(0, "f32")
    f.set_geometry(geo)
    f.set_hamiltonian(dataclasses.replace(w.hamiltonian, ddi=3))
    ntrain, ntest = 600, 24
    tex = torch.tensor(bench.film_textures(geo, ntrain + ntest, 2024), device="cuda").contiguous()
    bench.relax_textures(f, tex)
    lab = torch.zeros_like(tex)
    torch.cuda.synchronize()
    e.ddi_label_dev(ntrain + ntest, tex, lab)
    e.ddi_train_dev(ntrain, tex[:ntrain].contiguous(), lab[:ntrain].contiguous(), epochs=30, batch=8, lr=2e-3,
                    seed=0)
    test = tex[ntrain:].contiguous()
    with_net, without = torch.zeros_like(test), torch.zeros_like(test)
    e.ddi_forward_dev(ntest, test, with_net)
    e.ddi_backbone_dev(ntest, test, without)
    e.synchronize()
    wn, wo = with_net.cpu().numpy().astype(np.float64), without.cpu().numpy().astype(np.float64)
    spins = test.cpu().numpy().astype(np.float64)
    s = _oracle_system(ora, geo)
    rng = np.random.default_rng(8)
    err_w, err_o = [], []
    for b in range(ntest):
        sites = np.sort(rng.choice(geo.n_sites, 256, replace=False))
        exact = s.dipole_gradient_sites(spins[b], sites)
        nrm = np.linalg.norm(exact)
        err_w.append(np.linalg.norm(wn[b][:, sites] - exact) / nrm)
        err_o.append(np.linalg.norm(wo[b][:, sites] - exact) / nrm)
    err_w, err_o = np.array(err_w), np.array(err_o)
    print(f"[residual] 128x128x4 held-out error vs FP64 oracle: with network mean {err_w.mean():.2e} "
          f"max {err_w.max():.2e}; backbone alone mean {err_o.mean():.2e} max {err_o.max():.2e}; "
          f"below 1e-3: {int((err_w < 1e-3).sum())}/{ntest} with, {int((err_o < 1e-3).sum())}/{ntest} without",
          flush=True)
    assert err_w.mean() < (2.0 / 3.0) * err_o.mean()
    e.close()
    f.close()


def test_llg_with_the_learned_field_follows_the_direct_sum():
    """A trained residual network behind the residual check (tol 1e-3, 256
    sites) in 20 LLG steps of the 64 x 64 x 4 film: some evaluations pass the
    check without the direct sum, and the spins stay as close to the
    direct-sum trajectory as a field error of twice the tolerance allows:
    per step the rotation differs by at most gamma (1 + alpha) / (1 +
    alpha^2) |dB| dt with |dB| <= 2 tol max|B_dd| (B_dd in Tesla from the
    direct sum at the start), summed over the steps."""
    import torch

    import paper_1901_11350_amd as pk

    announce("residual LLG with check")
    geo = _film()
    e = _engine(geo, seed=6)
    tex = np.stack([_f32(_texture(geo, k)) for k in range(240)])
    nt = torch.tensor(tex, dtype=torch.float32, device="cuda").contiguous()
    lab = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_label_dev(240, nt, lab)
    e.ddi_train_dev(240, nt, lab, epochs=40, batch=8, lr=2e-3, seed=0)
    n0 = _texture(geo, 1000 + 2)
    e.set_hamiltonian(dataclasses.replace(HAM4, ddi=2))
    e.ddi_configure(1e-3, 256)
    e.set_spins(n0)
    e.run(0.3, 0.001, 20)
    st = e.ddi_stats()
    got = e.get_spins()
    d = pk.Engine(0, "f32")
    d.set_geometry(geo)
    d.set_hamiltonian(dataclasses.replace(HAM4, ddi=True))
    d.set_spins(n0)
    d.run(0.3, 0.001, 20)
    ref = d.get_spins()
    d.set_spins(n0)
    bdd = np.linalg.norm(d.dipole_gradient(), axis=0).max() / (HAM4.mu[0] * 0.057883818060)
    alpha, dt, gamma = 0.3, 0.001, 0.176085963023
    bound = 20 * gamma * (1 + alpha) / (1 + alpha ** 2) * (2 * 1e-3 * bdd) * dt
    print(f"[residual] LLG: {st['evaluations']} evaluations, {st['fallbacks']} fallbacks, last sampled error "
          f"{st['last_error']:.2e}, max {st['max_error']:.2e}; max spin difference {np.abs(got - ref).max():.2e} "
          f"(bound {bound:.2e}, max |B_dd| {bdd:.2f} T)", flush=True)
    assert st["evaluations"] == 40 and st["fallbacks"] < st["evaluations"]
    assert np.abs(got - ref).max() < bound
    e.close()
    d.close()
