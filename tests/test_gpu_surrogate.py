"""GPU tests of the learned dipole-field surrogate: matrix-core convolution
forward and backward against the FP64 oracle (same bf16 contract), the
forward against the oracle's exact network within a derived bf16 bound,
training lowers the loss, and the residual check's fallback reproduces the
direct sum exactly."""

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


U_BF16 = 2.0 ** -8          # unit roundoff of bfloat16 (8 significant bits)
U_F32 = 2.0 ** -24
SILU_LIP = 1.0998           # max |d silu / dz|
SILU_REL = 2.0 ** -18       # relative error allowed to the FP32 silu (exp, divide)


def _bf16_network_bound(ora, ws, bs, x):
    """Elementwise a-priori bound on |GPU network - exact network| for an
    input x (FP64), derived layer by layer from the kernel's arithmetic:
    the input and every weight are rounded to FP32 and then bf16 (relative
    error u' = u + 2^-23 each), products of bf16 values are exact in FP32 and
    summed over K = 9 x 32 terms in FP32 (gamma_K), the bias is FP32, a
    hidden activation is the FP32 silu (relative error 2^-18) rounded to bf16
    (u).  With e the bound on the layer's input error and a its exact input,
    the pre-activation error is
        u' conv(|a| + e, |w|) + conv(e, |w|) + gamma_K (1 + u') conv(|a| + e, |w|)
        + 2^-24 (|b| + |z| + e_z)
    and the next input error L e_z + (u + 2^-18)(|silu(z)| + L e_z), L the
    Lipschitz constant of silu; the last layer's output is FP32 (2^-24).
    conv(., |w|) is the oracle's exact convolution of absolute values."""
    u1 = U_BF16 + 2 * U_F32
    gam = (9 * 32 + 2) * U_F32 / (1 - (9 * 32 + 2) * U_F32)
    a = np.asarray(x, dtype=np.float64)
    e = u1 * np.abs(a)
    with ora.conv_exact():
        for k, (w, b) in enumerate(zip(ws, bs)):
            zero = np.zeros(w.shape[3])
            aw = ora.conv3x3_fwd(np.abs(a) + e, np.abs(w), zero)
            ew = ora.conv3x3_fwd(e, np.abs(w), zero)
            z = ora.conv3x3_fwd(a, w, b)
            ez = u1 * aw + ew + gam * (1 + u1) * aw
            ez = ez + U_F32 * (np.abs(b) + np.abs(z) + ez)
            if k + 1 == len(ws):
                return z, ez + U_F32 * (np.abs(z) + ez)
            y = ora.silu(z)[0]
            e = SILU_LIP * ez + (U_BF16 + SILU_REL) * (np.abs(y) + SILU_LIP * ez)
            a = y


def _rounding_model_net(ora, ws, bs, x, rng):
    """The exact network with every operand the kernel rounds (input, each
    weight, each stored hidden activation) multiplied by an independent
    1 + eps, eps uniform in [-u, u]: the random-rounding model of bf16."""
    def pert(a):
        return a * (1 + rng.uniform(-U_BF16, U_BF16, a.shape)) if rng is not None else a
    a = pert(x)
    with ora.conv_exact():
        for k, (w, b) in enumerate(zip(ws, bs)):
            z = ora.conv3x3_fwd(a, pert(w), b)
            if k + 1 == len(ws):
                return z
            a = pert(ora.silu(z)[0])


def _forward_against_exact(ora, channels, seed):
    import torch

    geo = _film()
    e = _engine(geo)
    e.ddi_init(channels, seed=7)
    n_p = sum(9 * a * b + b for a, b in zip(channels[:-1], channels[1:]))
    p = np.random.default_rng(seed).standard_normal(n_p) * 0.15
    e.ddi_set_params(p)
    n = np.stack([si.uniform_sphere(geo.n_sites, seed + 3),
                  si.skyrmion_ansatz(geo, radius=7.0, noise_rad=0.2, seed=seed + 4)])
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    ft = torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_forward_dev(2, nt, ft)
    e.synchronize()
    e.close()
    got = ft.cpu().numpy().astype(np.float64)
    ws, bs = _params_to_layers(p, channels)
    x = _to_nhwc(geo, n.astype(np.float32).astype(np.float64))
    return geo, got, ws, bs, x


def test_one_layer_forward_within_the_rigorous_bf16_bound(ora):
    """One 3x3 layer with parameters and spins that are not bf16-exact,
    against the oracle's exact (unrounded FP64) layer: every output within
    the elementwise bound derived above from the kernel's arithmetic."""
    announce("surrogate one layer vs exact, rigorous bound")
    geo, got, ws, bs, x = _forward_against_exact(ora, [12, 12], 55)
    z, ez = _bf16_network_bound(ora, ws, bs, x)
    scale = C_DD * HAM4.mu[0] ** 2
    ref = _field_from_nhwc(geo, z) * scale
    bound = _field_from_nhwc(geo, ez) * scale * (1 + 4 * U_F32) + 1e-30
    ratio = (np.abs(got - ref) / bound).max()
    print(f"[surrogate] one layer: max |dev|/bound {ratio:.3f}, normwise error {np.linalg.norm(got - ref) / np.linalg.norm(ref):.3e}, "
          f"normwise bound {np.linalg.norm(bound) / np.linalg.norm(ref):.3e}", flush=True)
    assert ratio <= 1.0
    assert np.linalg.norm(bound) <= 0.1 * np.linalg.norm(ref)


def test_four_layer_forward_within_the_bf16_rounding_model(ora):
    """The 4-layer 32-channel network (parameters and spins not bf16-exact)
    against the oracle's exact FP64 network.  Worst-case bounds compound
    through four layers of 288-term sums to far above the field itself, so
    the bar is the random-rounding model: the normwise error of the engine
    must not exceed 1.5 times the largest of four oracle runs of the exact
    network with every rounded operand perturbed by an independent relative
    error uniform in [-u, u] (u = 2^-8)."""
    channels = [12, 32, 32, 32, 12]
    announce(f"surrogate forward vs exact network {channels}")
    geo, got, ws, bs, x = _forward_against_exact(ora, channels, 77)
    z = _rounding_model_net(ora, ws, bs, x, None)
    model = max(np.linalg.norm(_rounding_model_net(ora, ws, bs, x, np.random.default_rng(1000 + k)) - z)
                / np.linalg.norm(z) for k in range(4))
    ref = _field_from_nhwc(geo, z) * C_DD * HAM4.mu[0] ** 2
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"[surrogate] four layers: normwise error {err:.3e}, rounding model {model:.3e}", flush=True)
    assert err <= 1.5 * model
    assert model < 0.05


def test_small_grid_tiles_equal_full_tiles():
    """A small grid runs the convolutions on 16 x 4 pixel tiles (four times
    the workgroups), a large batch on 16 x 16 tiles; same taps and
    instructions per accumulator, so the outputs agree bit for bit (64 x 64
    film: one sample takes the small tiles, four samples the full ones)."""
    import torch

    channels = [12, 32, 32, 32, 12]
    announce("conv tiles 16x4 vs 16x16")
    geo = _film(64)
    e = _engine(geo)
    e.ddi_init(channels, seed=9)
    n_p = sum(9 * a * b + b for a, b in zip(channels[:-1], channels[1:]))
    e.ddi_set_params(np.random.default_rng(99).standard_normal(n_p) * 0.15)
    n = np.stack([si.uniform_sphere(geo.n_sites, 91 + k) for k in range(4)])
    nt = torch.tensor(n, dtype=torch.float32, device="cuda").contiguous()
    batch, single = torch.zeros_like(nt), torch.zeros_like(nt)
    torch.cuda.synchronize()
    e.ddi_forward_dev(4, nt, batch)
    for b in range(4):
        e.ddi_forward_dev(1, nt[b].contiguous(), single[b])
    e.synchronize()
    e.close()
    assert torch.equal(batch, single)
    assert float(batch.abs().max()) > 0


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
