"""GPU tests of the learned dipole-field surrogate: matrix-core convolution
forward and backward against the FP64 oracle (same bf16 contract), training
lowers the loss, and the residual check's fallback reproduces the direct
sum exactly."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, need_gpu, rel_err

pytestmark = pytest.mark.gpu

HAM4 = si.WORKLOADS["film128x4_dipolar"].hamiltonian
C_DD = 1.00000000055e-7 * 9.2740100783e-24 ** 2 / 1e-30 / 1.602176634e-22


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _film(L=32, layers=4):
    return si.simple_cubic(L, L, layers, periodic=(0, 0, 0))


def _engine(geo, mode=1):
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, "f32")
    e.set_geometry(geo)
    e.set_hamiltonian(dataclasses.replace(HAM4, ddi=True))
    return e


def _samples(ora, geo, count, seed):
    """bf16-exact spin samples (rounded on the host) -> (count, 3, N)."""
    out = []
    for k in range(count):
        if k % 2 == 0:
            n = si.uniform_sphere(geo.n_sites, seed + k)
        else:
            n = si.skyrmion_ansatz(geo, radius=6.0 + k, noise_rad=0.2, seed=seed + k)
        out.append(ora.bf16(n))
    return np.stack(out)


def _to_nhwc(geo, n):
    """(B, 3, N) film spins -> (B, H, W, 3*layers) in the network's channel order."""
    W, H, L = geo.n_cells
    B = n.shape[0]
    x = n.reshape(B, 3, L, H, W)            # comp, layer, y, x
    return x.transpose(0, 3, 4, 2, 1).reshape(B, H, W, 3 * L)


def _params_to_layers(p, ch):
    ws, bs, q = [], [], 0
    for k in range(len(ch) - 1):
        nw = 9 * ch[k] * ch[k + 1]
        ws.append(p[q:q + nw].reshape(3, 3, ch[k], ch[k + 1]))
        q += nw
        bs.append(p[q:q + ch[k + 1]])
        q += ch[k + 1]
    return ws, bs


def _field_from_nhwc(geo, y):
    W, H, L = geo.n_cells
    B = y.shape[0]
    return y.reshape(B, H, W, L, 3).transpose(0, 4, 3, 1, 2).reshape(B, 3, L * H * W)


def _seeded_params(ora, channels, seed, scale=0.15):
    """bf16-exact parameters from a seeded NumPy generator."""
    n = sum(9 * a * b + b for a, b in zip(channels[:-1], channels[1:]))
    return ora.bf16(np.random.default_rng(seed).standard_normal(n) * scale)


def _oracle_dipole(ora, geo, n):
    """FP64 dipole gradient (meV) of each sample from the oracle."""
    ham = si.Hamiltonian(mu=HAM4.mu, B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), ddi=True)
    s = ora.System(geo, ham)
    return np.stack([s.gradient(n[b]) for b in range(n.shape[0])])


@pytest.mark.parametrize("channels", [[12, 12], [12, 32, 32, 32, 12]])
def test_surrogate_forward_matches_oracle(ora, channels):
    import torch

    announce(f"surrogate forward {channels}")
    geo = _film()
    e = _engine(geo)
    e.ddi_init(channels, seed=3)
    p = _seeded_params(ora, channels, 33)
    e.ddi_set_params(p)
    n = _samples(ora, geo, 3, 40)
    mu = HAM4.mu[0]
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    ft = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_forward_dev(3, nt, ft)
    e.synchronize()
    got = ft.cpu().numpy().astype(np.float64)
    ws, bs = _params_to_layers(p, channels)
    ref = _field_from_nhwc(geo, ora.SurrogateNet(ws, bs).forward(_to_nhwc(geo, n))) * C_DD * mu * mu
    # One layer: the only difference is FP32 versus FP64 accumulation of
    # bf16-exact products.  Several layers: each hidden activation is rounded
    # to bf16 on both sides, and an accumulation difference of ~1e-6 next to
    # a rounding boundary moves that activation by one bf16 ulp (2^-8
    # relative); such flips spread through the following layers, so the
    # normwise bound is one bf16 ulp.
    tol = 1e-5 if len(channels) == 2 else 2.0 ** -8
    assert rel_err(got, ref) <= tol


def test_surrogate_gradients_match_oracle(ora):
    import torch

    announce("surrogate gradients")
    channels = [12, 16, 16, 12]
    geo = _film()
    e = _engine(geo)
    e.ddi_init(channels, seed=5)
    p = _seeded_params(ora, channels, 55)
    e.ddi_set_params(p)
    n = _samples(ora, geo, 2, 50)
    labels = _oracle_dipole(ora, geo, n)
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    lab = torch.tensor(labels, dtype=torch.float32, device="cuda").contiguous()
    torch.cuda.synchronize()
    loss, g = e.ddi_loss_grad_dev(2, nt, lab)
    ws, bs = _params_to_layers(p, channels)
    mu = HAM4.mu[0]
    target = _to_nhwc(geo, labels / (C_DD * mu * mu))
    lo, gw, gb = ora.SurrogateNet(ws, bs).loss_and_grads(_to_nhwc(geo, n), target)
    assert loss == pytest.approx(lo, rel=1e-4)
    gws, gbs = _params_to_layers(g, channels)
    for k in range(len(channels) - 1):
        assert rel_err(gws[k], gw[k]) <= 2e-3, k
        assert rel_err(gbs[k], gb[k]) <= 2e-3, k


def test_training_lowers_the_loss():
    import torch

    announce("surrogate training")
    geo = _film()
    e = _engine(geo)
    e.ddi_init([12, 32, 32, 32, 12], seed=1)
    n = np.stack([si.skyrmion_ansatz(geo, radius=4.0 + k, noise_rad=0.1, seed=k) if k % 2 else
                  si.domain_walls(geo, n_walls=1 + k % 3, seed=k) for k in range(16)])
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    lab = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_label_dev(16, nt, lab)
    losses = e.ddi_train_dev(16, nt, lab, epochs=30, batch=4, lr=2e-3, seed=0)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]


def test_fallback_reproduces_direct_sum_exactly():
    """Untrained network, tolerance 1e-3: every evaluation fails the residual
    check and the direct sum replaces it, so the LLG trajectory is the
    direct-sum trajectory bit for bit."""
    import paper_1901_11350_amd as pk

    announce("surrogate fallback")
    geo = _film()
    n0 = si.skyrmion_ansatz(geo, radius=6.0, noise_rad=0.2, seed=2)
    runs = {}
    for mode in (1, 2):
        e = pk.Engine(0, "f32")
        e.set_geometry(geo)
        e.set_hamiltonian(dataclasses.replace(HAM4, ddi=True))
        if mode == 2:
            e.ddi_init([12, 32, 32, 32, 12], seed=9)
            e.set_hamiltonian(dataclasses.replace(HAM4, ddi=2))
            e.ddi_configure(1e-3, 256)
        e.set_spins(n0)
        e.run(0.3, 0.001, 5)
        runs[mode] = e.get_spins()
        if mode == 2:
            st = e.ddi_stats()
            assert st["evaluations"] == 10 and st["fallbacks"] == 10
    assert np.array_equal(runs[1], runs[2])
