"""Benchmark: LLG spin-updates/s of the fused Depondt step on one MI355X.

Workload (default, the largest single-GPU configuration): simple-cubic
lattice 128^3 (2,097,152 spins), periodic, exchange J1 = 1.0 and J2 = 0.1
meV, bulk DMI 0.15 meV on the first shell, B = 0.3 T, T = 0, alpha = 0.5,
dt = 1 fs, FP32 spins, FP64 observables every 100 steps, from a seeded
conical spiral.  A "step" is one full Depondt step (predictor + corrector)
of every spin.  The same run also reports, each in a few seconds, the
stochastic 512^2 triangular workload, the 96-replica batch with its GNEB
chain, the stand-alone stencil on the 8192^2 probe lattice, and the dipole
field of the 128x128x4 film (direct sum, FFT convolution, learned field
with its residual check); --no-extras leaves them out.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_UPDATE = {"f32": 24.0, "f64": 48.0}   # read n, write n(t+dt): 3 components each
# Non-packed VALU issue capacity of MI355X: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 3.93e13 lane-instructions/s (one wave64 instruction per SIMD
# every four cycles).  This build emits no packed-FP32 instructions.
VALU_LANE_INSTR_PER_S = 256 * 64 * 2.4e9

KERNEL_SOURCES = {
    "k_fused2d_shape": ["paper_1901_11350_amd/csrc/kernels_fused2d.hpp",
                        "paper_1901_11350_amd/csrc/kernels_field.hpp",
                        "paper_1901_11350_amd/csrc/device_common.hpp"],
    "k_fused3d_shape": ["paper_1901_11350_amd/csrc/kernels_fused3d.hpp",
                        "paper_1901_11350_amd/csrc/kernels_fused2d.hpp",
                        "paper_1901_11350_amd/csrc/kernels_field.hpp",
                        "paper_1901_11350_amd/csrc/device_common.hpp"],
}


def kernel_source_digest(kernel: str) -> str:
    import hashlib

    h = hashlib.sha256()
    for p in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record(kernel: str, workload: str, step_path: str):
    """The committed rocprofv3 counter record of this kernel, workload and
    step path (profiles/counters_<kernel>_<workload>.json: FETCH_SIZE and
    WRITE_SIZE scaled by a device copy, VALU instructions per update), or
    None when there is none or the kernel sources changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_digest(kernel) or rec.get("step_path") != step_path:
        return None
    return rec


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(workload, budget_s: float = 12.0) -> dict:
    """The FP64 oracle, as it stands, on the host cores: Depondt steps of the
    same workload until about budget_s seconds of CPU work have been spent."""
    import oracle
    import spin_inputs as si

    oracle.build(force=False)
    w = workload
    s = oracle.System(w.geometry, w.hamiltonian)
    n = initial_state(w)
    d = w.dynamics
    steps = 0
    t0 = time.perf_counter()
    while True:
        n, _ = s.run(n, d.alpha, d.dt, 1, T=d.T, seed=d.seed, step0=steps)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 2000:
            break
    cores = oracle.num_threads()
    out = {"value": s.N * steps / el, "unit": "spin-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} FP64 Depondt steps of the full {s.N}-spin workload ({el:.1f} s)",
           "host": host_info()}
    # the same oracle on one core (the paper compares one thread with many)
    oracle.set_num_threads(1)
    try:
        steps1 = 0
        t0 = time.perf_counter()
        while True:
            n, _ = s.run(n, d.alpha, d.dt, 1, T=d.T, seed=d.seed, step0=steps + steps1)
            steps1 += 1
            el1 = time.perf_counter() - t0
            if el1 >= budget_s / 2 or steps1 >= 2000:
                break
    finally:
        oracle.set_num_threads(cores)
    out["single_core"] = {"value": s.N * steps1 / el1, "cores": 1,
                          "sample": f"{steps1} steps ({el1:.1f} s)"}
    return out


def initial_state(w):
    import spin_inputs as si

    if w.init == "conical_helix":
        return si.conical_helix(w.geometry, seed=w.init_seed)
    return si.uniform_sphere(w.geometry.n_sites, w.init_seed)


def calibrate_copy(mib: int, reps: int = 5) -> None:
    """A plain device-to-device copy of known size: the reference that HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) are scaled against."""
    import torch

    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 4 * n,
                      "bytes_written_per_launch": 4 * n, "ms_per_launch": ms,
                      "GBps": 8 * n / (ms * 1e-3) / 1e9}), flush=True)


_STREAM = None


def work_stream():
    """One dedicated (non-default, default-priority) stream: the engines
    launch every kernel on it and the timing events are recorded on it."""
    global _STREAM
    import torch

    if _STREAM is None:
        _STREAM = torch.cuda.Stream()
        assert _STREAM.cuda_stream != 0
    return _STREAM


def bench_batch(args) -> dict:
    """96 replicas (sides from {32, 64, 128, 256}, T uniform in 0-100 K, the
    square32 Hamiltonian, FP32) advanced as one batch, against the same
    replicas advanced one engine at a time."""
    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si
    from spin_inputs.workloads import batch_replica_table

    table = batch_replica_table(96, 11353)
    ham = si.WORKLOADS["square32_fp64"].hamiltonian
    alpha, dt, seed = 0.3, 0.001, 11353
    stream = work_stream()
    b = pk.Batch(0, stream=stream)
    engines = []
    for r, (L, T) in enumerate(table):
        e = pk.Engine(0, "f32", stream=stream)
        e.set_geometry(si.square(L, L))
        e.set_hamiltonian(ham)
        e.set_spins(si.uniform_sphere(e.N, 20000 + r))
        b.add(e, alpha, dt, T=T, seed=seed, replica=r)
        engines.append((e, T, r))
    total = sum(L * L for L, _ in table)
    b.set_chunk(args.batch_chunk)
    tuned = b.autotune(8)
    b.run(args.batch_chunk)
    torch.cuda.synchronize()
    K = args.batch_steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.run(K)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # the same replicas, one engine (one launch per step each) at a time
    Ks = max(10, K // 10)
    for e, T, r in engines:
        e.run(alpha, dt, 2, T=T, seed=seed, replica=r)
    torch.cuda.synchronize()
    ev0.record(stream)
    for e, T, r in engines:
        e.run(alpha, dt, Ks, T=T, seed=seed, replica=r)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_sep = ev0.elapsed_time(ev1)
    n_res = sum(1 for r in range(len(table)) if b.info(r)[1])
    # the 32-image GNEB chain on a 128x128 lattice (same Hamiltonian), FP32
    geo = si.square(128, 128)
    ge = pk.Engine(0, "f32", stream=stream)
    ge.set_geometry(geo)
    ge.set_hamiltonian(ham)
    a = si.skyrmion_ansatz(geo, radius=5.0, width=1.5)
    chain = si.geodesic_chain(a, si.ferromagnet(geo.n_sites, (0, 0, 1)), 32, fallback_axis=(1, 0, 0))
    g = pk.Gneb(ge, chain, k_spring=1.0, vp_dt=0.1)
    g.iterate(20)
    torch.cuda.synchronize()
    ev0.record(stream)
    g.iterate(args.gneb_iters)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_gneb = ev0.elapsed_time(ev1) / args.gneb_iters
    gneb = {"images": 32, "spins_per_image": geo.n_sites, "ms_per_iteration": ms_gneb,
            "image_spin_updates_per_s": 32 * geo.n_sites / (ms_gneb * 1e-3)}
    # the chain attached to the batch: one VP iteration per batch step, its
    # chunk graph launched beside the replicas' on the batch's side stream
    b.add_gneb(g)
    b.run(args.batch_chunk)
    torch.cuda.synchronize()
    ev0.record(stream)
    b.run(K)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_both = ev0.elapsed_time(ev1)
    gneb["in_batch"] = {"ms_per_step": ms_both / K,
                        "updates_per_s": (total + 32 * geo.n_sites) * K / (ms_both * 1e-3),
                        "note": "replica spin-updates + chain image-spin updates per second; the chain's graph runs beside the replicas' graph"}
    b.close()
    g.close()
    ge.close()
    for e, _, _ in engines:
        e.close()
    return {"workload": "batch96_square", "replicas": len(table), "resident_replicas": n_res, "gneb": gneb,
            "total_spins": total, "steps": K, "chunk": args.batch_chunk,
            "spin_updates_per_s": total * K / (ms * 1e-3), "ms_per_step": ms / K,
            "separate_engines_spin_updates_per_s": total * Ks / (ms_sep * 1e-3),
            "batch_gain": (total * K / ms) / (total * Ks / ms_sep), "autotune_ms_per_step": tuned}


def bench_stencil(args) -> dict:
    """The stand-alone stencil field kernel (sp_gradient_dev: exchange, DMI,
    anisotropy, Zeeman from LDS-staged tiles) on the 512^2 triangular
    workload and on the 8192^2 probe lattice, whose working set exceeds the
    last-level cache; algorithmic HBM bytes 24 per site (read n, write g)."""
    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si

    out = {}
    stream = work_stream()
    for name in ("triangular512_sllg", "square8192_probe"):
        w = si.WORKLOADS[name]
        e = pk.engine_for(w, 0, "f32", stream=stream)
        e.set_spins(si.uniform_sphere(e.N, w.init_seed))
        g = torch.empty((3, e.N), dtype=torch.float32, device="cuda")
        for _ in range(3):
            e.gradient_dev(g)
        torch.cuda.synchronize()
        K = args.stencil_launches
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(K):
            e.gradient_dev(g)
        ev1.record(stream)
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) * 1e-3 / K
        gbps = 24.0 * e.N / t / 1e9
        out[name] = {"n_sites": e.N, "us_per_launch": t * 1e6, "hbm_gbps_algorithmic": gbps,
                     "hbm_frac": gbps / HBM_PEAK_GBPS, "kernel": "k_gradient_shape", "launches": K}
        if name == "square8192_probe":
            # a device copy of the same bytes (read 12 B, write 12 B per site): the
            # practical HBM ceiling the stencil is measured against
            src = torch.empty((3, e.N), dtype=torch.float32, device="cuda")
            with torch.cuda.stream(stream):
                for _ in range(3):
                    g.copy_(src)
                ev0.record(stream)
                for _ in range(K):
                    g.copy_(src)
                ev1.record(stream)
            torch.cuda.synchronize()
            tc = ev0.elapsed_time(ev1) * 1e-3 / K
            out[name]["copy_same_bytes_gbps"] = 24.0 * e.N / tc / 1e9
            out[name]["frac_of_copy"] = gbps / out[name]["copy_same_bytes_gbps"]
            del src
        e.close()
        del g, e
        torch.cuda.empty_cache()
    # a lattice with a basis beyond the last-level cache: the honeycomb
    # (three shells, interfacial DMI) of 4096 x 2048 cells, 16.8M spins, on
    # the LDS-tiled field of the fused tile path
    w = basis_workloads()[0]
    e = pk.Engine(0, "f32", stream=stream)
    e.set_geometry(w.geometry.with_cells((4096, 2048, 1)))
    e.set_hamiltonian(w.hamiltonian)
    e.set_spins_dev(torch.nn.functional.normalize(
        torch.randn((3, e.N), generator=torch.Generator().manual_seed(5)), dim=0).to("cuda"))
    g = torch.empty((3, e.N), dtype=torch.float32, device="cuda")
    for _ in range(3):
        e.gradient_dev(g)
    torch.cuda.synchronize()
    K = args.stencil_launches
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(K):
        e.gradient_dev(g)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) * 1e-3 / K
    gbps = 24.0 * e.N / t / 1e9
    out["honeycomb4096x2048_probe"] = {"n_sites": e.N, "us_per_launch": t * 1e6, "hbm_gbps_algorithmic": gbps,
                                       "hbm_frac": gbps / HBM_PEAK_GBPS, "kernel": "k_gradient_tile",
                                       "launches": K, "step_path": e.step_path}
    e.close()
    del g, e
    torch.cuda.empty_cache()
    return out


def basis_workloads():
    """Lattices with a basis at about 262,144 spins (FP32, T = 10 K): the
    honeycomb with three exchange shells and interfacial DMI, the kagome
    lattice with two, and the two-atom (bcc) cell in 3D."""
    import spin_inputs as si

    hc = si.Hamiltonian(mu=(2.0, 2.5), B=(0.1, -0.2, 0.5), K=(0.1, 0.05),
                        K_axis=((0, 0, 1), (0.6, 0.0, 0.8)), J=(1.0, 0.2, -0.1), D=(0.15,))
    kg = si.Hamiltonian(mu=(2.0, 2.0, 3.0), B=(0.0, 0.0, 0.4), K=(0.1, 0.1, 0.2),
                        K_axis=((0, 0, 1),) * 3, J=(1.0, -0.2), D=(0.1,))
    bcc = si.Hamiltonian(mu=(2.0, 3.0), B=(0.2, 0.4, -0.3), K=(0.1, -0.2),
                         K_axis=((0, 0, 1), (0.6, 0.8, 0.0)), J=(1.0, 0.5), D=(0.1, 0.05), dmi_kind=si.DMI_BULK)
    bcc_geo = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.5, 0.5, 0.5)),
                          (64, 64, 32), (1, 1, 1))
    dyn = si.Dynamics(alpha=0.1, dt=0.0005, T=10.0, seed=3)
    return [si.Workload("honeycomb512x256", si.honeycomb(512, 256), hc, dyn, "f32", "uniform", 5,
                        "honeycomb 512x256 (2 atoms), J1-J3, interfacial D"),
            si.Workload("kagome512x171", si.kagome(512, 171), kg, dyn, "f32", "uniform", 6,
                        "kagome 512x171 (3 atoms), J1-J2, interfacial D"),
            si.Workload("bcc64x64x32", bcc_geo, bcc, dyn, "f32", "uniform", 7,
                        "two-atom cubic cell 64x64x32, J1-J2, bulk D")]


def bench_basis(args) -> dict:
    """Lattices with a basis: the fused tile step (one launch, 24 B per
    FP32 spin-update) against the two-pass kernels (60 B) per step."""
    out = {}
    for w in basis_workloads():
        res = {}
        for path in ("fusedtile", "twopass"):
            r = time_workload(w, args.basis_steps, 20, 0, step_path=path)
            res[path] = r
        ft = res["fusedtile"]
        out[w.name] = {"n_sites": ft["N"], "steps": args.basis_steps,
                       "us_per_step_fusedtile": ft["ms"] * 1e3 / ft["steps"],
                       "us_per_step_twopass": res["twopass"]["ms"] * 1e3 / res["twopass"]["steps"],
                       "spin_updates_per_s": ft["N"] * ft["steps"] / (ft["ms"] * 1e-3),
                       "hbm_gbps_algorithmic": BYTES_PER_UPDATE["f32"] * ft["N"] / ft["t_launch"] / 1e9,
                       "speedup": res["twopass"]["ms"] / ft["ms"], "description": w.description}
    return out


def film_textures(geo, count: int, seed: int):
    """Seeded training/test textures of the dipolar film: a third uniform
    random, a third 1-3 tanh domain walls (Bloch or Neel, random position,
    orientation and width 2-8 a), a third skyrmion/bubble ansatz (radius
    5-20 a, random centre and helicity, small tilt noise) that
    relax_textures relaxes on the GPU."""
    import numpy as np

    import spin_inputs as si

    rng = np.random.default_rng(seed)
    out = np.empty((count, 3, geo.n_sites), dtype=np.float32)
    W, H, _ = geo.n_cells
    for k in range(count):
        kind = k % 3
        s = int(rng.integers(1 << 30))
        if kind == 0:
            n = si.uniform_sphere(geo.n_sites, s)
        elif kind == 1:
            n = si.domain_walls(geo, n_walls=int(rng.integers(1, 4)), seed=s, bloch=bool(rng.integers(2)))
        else:
            n = si.skyrmion_ansatz(geo, radius=float(rng.uniform(5, 20)),
                                   center=(float(rng.uniform(0.25, 0.75) * W), float(rng.uniform(0.25, 0.75) * H)),
                                   helicity=float(rng.uniform(0, 6.283)), width=float(rng.uniform(1.5, 4.0)),
                                   noise_rad=0.05, seed=s)
        out[k] = n
    return out


def relax_textures(engine, tex, steps: int = 200, alpha: float = 0.5):
    """Relax every third texture (the skyrmion/bubble ansatz) in place by
    `steps` damped Depondt steps (T = 0, dt = 1 fs) of the film's full
    Hamiltonian on the GPU (dipole field by the FFT convolution, the same
    pair sum as the direct sum)."""
    for k in range(2, tex.shape[0], 3):
        engine.set_spins_dev(tex[k])
        engine.run(alpha, 0.001, steps)
        engine.get_spins_dev(tex[k])


def bench_surrogate(args) -> dict:
    """Dipole field of the 128x128x4 film: the direct sum, the FFT
    convolution and the residual form of the learned field (exact near
    blocks + far block dipoles + a network trained on textures labelled by
    the direct sum), each per field and inside the LLG step; the learned
    field behind its residual check (tol 1e-3, 256 sampled sites) with its
    fallback rate; held-out errors against the FP32 direct sum with and
    without the network."""
    import dataclasses

    import numpy as np
    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si

    w = si.WORKLOADS["film128x4_dipolar"]
    geo = w.geometry
    stream = work_stream()
    e = pk.Engine(0, "f32", stream=stream)
    e.set_geometry(geo)
    e.set_hamiltonian(w.hamiltonian)
    f = pk.Engine(0, "f32", stream=stream)
    f.set_geometry(geo)
    f.set_hamiltonian(dataclasses.replace(w.hamiltonian, ddi=3))
    N = e.N
    ntr, nte = args.sur_train, args.sur_test
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    tex = torch.tensor(film_textures(geo, ntr + nte, 11354), device="cuda").contiguous()
    print(f"[bench] dipole: {ntr + nte} textures generated ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    with torch.cuda.stream(stream):
        relax_textures(f, tex)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    print(f"[bench] dipole: every third texture relaxed ({data_s:.1f} s)", file=sys.stderr, flush=True)
    lab = torch.zeros_like(tex)
    ev0.record(stream)
    e.ddi_label_dev(ntr + nte, tex, lab)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_direct = ev0.elapsed_time(ev1) / (ntr + nte)
    e.ddi_init_residual([12, 32, 32, 32, 12], seed=11354, block=4, reach=2)
    t0 = time.perf_counter()
    print(f"[bench] dipole: labels from the direct sum ({ms_direct:.3f} ms per field); training", file=sys.stderr,
          flush=True)
    losses = e.ddi_train_dev(ntr, tex[:ntr], lab[:ntr], epochs=args.sur_epochs, batch=8, lr=args.sur_lr, seed=1)
    train_s = time.perf_counter() - t0
    print(f"[bench] dipole: trained ({train_s:.1f} s)", file=sys.stderr, flush=True)
    test = tex[ntr:].contiguous()
    pred, base = torch.zeros_like(test), torch.zeros_like(test)
    e.ddi_forward_dev(nte, test, pred)
    e.ddi_backbone_dev(nte, test, base)
    torch.cuda.synchronize()

    def rel(a):
        return (torch.linalg.vector_norm((a - lab[ntr:]).reshape(nte, -1), dim=1) /
                torch.linalg.vector_norm(lab[ntr:].reshape(nte, -1), dim=1)).cpu().numpy()

    err, err_b = rel(pred), rel(base)
    # one field: the learned form (moments, backbone, network, correction)
    reps = 20
    ev0.record(stream)
    for _ in range(reps):
        e.ddi_forward_dev(1, test[:1], pred[:1])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_learned = ev0.elapsed_time(ev1) / reps
    ev0.record(stream)
    for _ in range(reps):
        e.ddi_backbone_dev(1, test[:1], base[:1])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_backbone = ev0.elapsed_time(ev1) / reps
    # LLG steps: direct sum, learned field behind the residual check, FFT
    # the workload's initial state: a bubble/skyrmion relaxed like the textures
    steps = args.sur_steps
    n0 = torch.tensor(si.skyrmion_ansatz(geo, radius=12.0, noise_rad=0.3, seed=w.init_seed), dtype=torch.float32,
                      device="cuda").reshape(1, 3, N).contiguous()
    three = torch.cat([n0, n0, n0]).contiguous()
    with torch.cuda.stream(stream):
        relax_textures(f, three)          # relaxes the third
    torch.cuda.synchronize()
    n0 = three[2].contiguous()
    out = {}
    for name, mode in (("direct", 1), ("learned", 2), ("fft", 3)):
        eng = f if mode == 3 else e
        if mode != 3:
            eng.set_hamiltonian(dataclasses.replace(w.hamiltonian, ddi=mode))
        if mode == 2:
            eng.ddi_configure(1e-3, 256)
        eng.set_spins_dev(n0)
        eng.run(0.3, 0.001, 2)
        before = eng.ddi_stats() if mode == 2 else None
        torch.cuda.synchronize()
        ev0.record(stream)
        eng.run(0.3, 0.001, steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        out[name] = ev0.elapsed_time(ev1) / steps
        if mode == 2:
            st = eng.ddi_stats()
            evals = st["evaluations"] - before["evaluations"]
            falls = st["fallbacks"] - before["fallbacks"]
            out["fallback_rate"] = falls / max(evals, 1)
            out["sampled_err_last"] = st["last_error"]
            out["sampled_err_max"] = st["max_error"]
    # FFT field on the held-out textures
    fft_pred = torch.zeros_like(test)
    f.dipole_gradient_dev(test[0], fft_pred[0])
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(nte):
        f.dipole_gradient_dev(test[k], fft_pred[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_fft = ev0.elapsed_time(ev1) / nte
    fft_err = rel(fft_pred)
    e.close()
    f.close()
    return {"workload": "film128x4_dipolar", "n_sites": N, "form": "residual (exact near blocks within 2 of 4x4x4 "
            "blocks, far block dipoles, 12-32-32-32-12 network on the 32x32 block grid)",
            "train_textures": ntr, "test_textures": nte, "relaxed_third_steps": 200, "data_s": data_s,
            "epochs": args.sur_epochs, "train_s": train_s, "loss_first_last": [float(losses[0]), float(losses[-1])],
            "heldout_rel_err_mean": float(err.mean()), "heldout_rel_err_max": float(err.max()),
            "heldout_rel_err_backbone_mean": float(err_b.mean()), "heldout_rel_err_backbone_max": float(err_b.max()),
            "heldout_below_tol": int((err < 1e-3).sum()), "heldout_backbone_below_tol": int((err_b < 1e-3).sum()),
            "ms_direct_sum_field": ms_direct, "ms_learned_field": ms_learned, "ms_backbone_field": ms_backbone,
            "field_speedup_learned": ms_direct / ms_learned, "direct_pairs_per_s": N * (N - 1) / (ms_direct * 1e-3),
            "ms_llg_step_direct": out["direct"], "ms_llg_step_learned": out["learned"],
            "step_speedup_learned": out["direct"] / out["learned"], "check_tol": 1e-3, "check_sites": 256,
            "fallback_rate": out["fallback_rate"], "sampled_err_last": out["sampled_err_last"],
            "sampled_err_max": out["sampled_err_max"],
            "ms_fft_field": ms_fft, "fft_rel_err_vs_direct_max": float(fft_err.max()),
            "field_speedup_fft": ms_direct / ms_fft, "ms_llg_step_fft": out["fft"],
            "step_speedup_fft": out["direct"] / out["fft"]}


def binder_table(precision, sizes, temps, therm, samples, method, seed=5):
    """U4 = 1 - <m^4>/(3 <m^2>^2) (m = |mean spin|) of the simple-cubic
    ferromagnet J = 1 meV, mu = 2, periodic L^3, from Metropolis sweeps
    (cone 60 deg) or stochastic Depondt LLG (alpha = 1, dt = 1 fs, one sample
    per 10 steps)."""
    import numpy as np

    import paper_1901_11350_amd as pk
    import spin_inputs as si

    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0,))
    out = {}
    for L in sizes:
        e = pk.Engine(0, precision, stream=work_stream())
        e.set_geometry(si.simple_cubic(L, L, L))
        e.set_hamiltonian(ham)
        for T in temps:
            e.set_spins(si.ferromagnet(e.N, (0, 0, 1)))
            if method == "mc":
                e.mc_run(T, 60.0, therm, seed=seed)
                obs, _ = e.mc_run(T, 60.0, samples, seed=seed, observe_every=1)
            else:
                e.run(1.0, 0.001, therm, T=T, seed=seed)
                obs = e.run(1.0, 0.001, 10 * samples, T=T, seed=seed, observe_every=10)
            m = np.array([np.linalg.norm(o["M"]) for o in obs])
            out[(L, T)] = float(1 - np.mean(m ** 4) / (3 * np.mean(m ** 2) ** 2))
    return out


def binder_crossing(u, L1, L2, temps):
    d = [u[(L1, T)] - u[(L2, T)] for T in temps]
    for k in range(len(temps) - 1):
        if d[k] < 0 <= d[k + 1]:
            return temps[k] + (temps[k + 1] - temps[k]) * (-d[k]) / (d[k + 1] - d[k])
    return None


def bench_tc(args) -> dict:
    """Critical temperature of the simple-cubic ferromagnet (J = 1 meV,
    expected 1.44 J/k_B = 16.71 K) from Binder-cumulant crossings: Metropolis
    with the paper's sampling (10k thermalisation + 100k samples per T) on
    L = 10, 16, 20, 30, and stochastic LLG on L = 8, 12 (shorter runs)."""
    temps = [15.5, 16.0, 16.5, 17.0, 17.5]
    t0 = time.perf_counter()
    mc = binder_table("f32", (10, 16, 20, 30), temps, args.tc_therm, args.tc_samples, "mc")
    t_mc = time.perf_counter() - t0
    t0 = time.perf_counter()
    llg = binder_table("f32", (8, 12), temps, args.tc_llg_therm, args.tc_llg_samples, "llg")
    t_llg = time.perf_counter() - t0
    pairs = [(10, 16), (16, 20), (20, 30)]
    return {"workload": "simple_cubic_ferromagnet_J1meV", "expected_K": 16.71, "temps_K": temps,
            "mc": {"sizes": [10, 16, 20, 30], "thermalisation_sweeps": args.tc_therm, "samples": args.tc_samples,
                   "U4": {f"L{L}_T{T}": v for (L, T), v in mc.items()},
                   "crossings_K": {f"{a}/{b}": binder_crossing(mc, a, b, temps) for a, b in pairs}, "s": t_mc},
            "llg": {"sizes": [8, 12], "thermalisation_steps": args.tc_llg_therm,
                    "samples_every_10_steps": args.tc_llg_samples,
                    "U4": {f"L{L}_T{T}": v for (L, T), v in llg.items()},
                    "crossing_K": binder_crossing(llg, 8, 12, temps), "s": t_llg}}


KERNEL_OF_PATH = {"fused2d": "k_depondt_fused2d", "fusedtile": "k_fused_tile", "twopass": "k_predict+k_correct", "shape3d": "k_fused3d_shape",
                  "persist2d": "k_persist2d", "shape2d": "k_fused2d_shape"}


def time_workload(w, steps: int, warmup: int, observe_every: int, step_path: str = "", autotune: bool = False):
    """Depondt steps of a workload between HIP events on the engine's stream:
    the whole run with its observations (the throughput), then the step
    kernel alone per launch (the roofline's achieved rate)."""
    import torch

    import paper_1901_11350_amd as pk

    d = w.dynamics
    stream = work_stream()
    e = pk.engine_for(w, 0, w.precision, stream=stream)
    try:
        e.set_spins(initial_state(w))
        tuned_ms = e.autotune(d.alpha, d.dt, d.T, d.seed, n_steps=50) if autotune else None
        if step_path:
            e.step_path = step_path
        print(f"[bench] workload={w.name} N={e.N} path={e.step_path} precision={w.precision} "
              f"autotune_ms={tuned_ms}", file=sys.stderr, flush=True)
        e.run(d.alpha, d.dt, warmup, T=d.T, seed=d.seed)
        torch.cuda.synchronize()
        K = steps
        oe = observe_every if observe_every and K >= observe_every else 0
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        ev0.record(stream)
        obs = e.run(d.alpha, d.dt, K, T=d.T, seed=d.seed, observe_every=oe)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = ev0.elapsed_time(ev1)
        # the step kernel alone (no observations), per launch; the persistent
        # path runs all steps in one launch, so its figure is per step
        K2 = max(100, K // 2)
        ev0.record(stream)
        e.run(d.alpha, d.dt, K2, T=d.T, seed=d.seed)
        ev1.record(stream)
        torch.cuda.synchronize()
        path = e.step_path
        launches_per_step = 2 if path == "twopass" else 1
        t_launch = ev0.elapsed_time(ev1) * 1e-3 / (K2 * launches_per_step)
        last = obs[-1] if obs else e.observe()
        return {"N": e.N, "steps": K, "observe_every": oe, "ms": ms, "wall_s": wall, "t_launch": t_launch,
                "launches_per_step": launches_per_step, "path": path, "last": last, "autotune_ms": tuned_ms}
    finally:
        e.close()


def roofline_of(w, r) -> dict:
    """HBM roofline of the step kernel: algorithmic bytes (24 B per FP32
    spin-update: read n, write n') per launch over its average launch time,
    against 8 TB/s; the VALU ceiling from the committed instruction count."""
    kernel = KERNEL_OF_PATH.get(r["path"].split("/")[0], "k_fused2d_shape")
    bytes_per_launch = BYTES_PER_UPDATE[w.precision] * r["N"] / r["launches_per_step"]
    achieved = bytes_per_launch / r["t_launch"] / 1e9
    rec = counter_record(kernel, w.name, r["path"])
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBPS,
           "traffic": (rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]) if rec else None,
           "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per_launch,
           "us_per_launch": r["t_launch"] * 1e6}
    if rec and rec.get("valu_instructions_per_update"):
        ipu = rec["valu_instructions_per_update"]
        ceiling = VALU_LANE_INSTR_PER_S / ipu
        upd = r["N"] / r["launches_per_step"] / r["t_launch"]
        out["valu"] = {"instructions_per_update": ipu, "lane_instructions_per_s_peak": VALU_LANE_INSTR_PER_S,
                       "ceiling_updates_per_s": ceiling, "achieved_updates_per_s": upd, "frac": upd / ceiling}
    return out


def bench_config1(args) -> dict:
    """The stochastic 512^2 triangular workload (T = 10 K), observations
    every 100 steps, graph-replayed chunks."""
    import spin_inputs as si

    w = si.WORKLOADS["triangular512_sllg"]
    r = time_workload(w, args.config1_steps, 200, 100)
    value = r["N"] * r["steps"] / (r["ms"] * 1e-3)
    return {"workload": w.name, "n_sites": r["N"], "steps": r["steps"], "ms_per_step": r["ms"] / r["steps"],
            "spin_updates_per_s": value, "step_path": r["path"], "roofline": roofline_of(w, r)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no config-1, batch, stencil, dipole keys)")
    ap.add_argument("--surrogate", action="store_true", help="(default with the extras; kept for old command lines)")
    ap.add_argument("--sur-train", type=int, default=1536)
    ap.add_argument("--sur-test", type=int, default=24)
    ap.add_argument("--sur-epochs", type=int, default=30)
    ap.add_argument("--sur-lr", type=float, default=2e-3)
    ap.add_argument("--sur-steps", type=int, default=20)
    ap.add_argument("--config1-steps", type=int, default=2000)
    ap.add_argument("--batch", action="store_true", help="(default with the extras; kept for old command lines)")
    ap.add_argument("--batch-steps", type=int, default=1024)
    ap.add_argument("--batch-chunk", type=int, default=32)
    ap.add_argument("--gneb-iters", type=int, default=1000)
    ap.add_argument("--basis", action="store_true", help="(default with the extras) lattices with a basis only")
    ap.add_argument("--basis-steps", type=int, default=500)
    ap.add_argument("--stencil", action="store_true", help="(default with the extras; kept for old command lines)")
    ap.add_argument("--stencil-launches", type=int, default=200)
    ap.add_argument("--tc", action="store_true",
                    help="also estimate the ferromagnet's Tc from Binder crossings (reported under 'tc')")
    ap.add_argument("--tc-therm", type=int, default=10000)
    ap.add_argument("--tc-samples", type=int, default=100000)
    ap.add_argument("--tc-llg-therm", type=int, default=20000)
    ap.add_argument("--tc-llg-samples", type=int, default=20000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run a device copy of this size (counter calibration)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cubic128_bulkdmi")
    ap.add_argument("--observe-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-path", default="",
                    help="force a step path (e.g. persist2d/32x16) instead of the engine's default")
    ap.add_argument("--autotune", action="store_true",
                    help="time every step path / tile shape first and keep the fastest (default: the engine's "
                         "default path, chosen from such sweeps)")
    ap.add_argument("--no-autotune", action="store_true", help="(default; kept for old command lines)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si

    w = si.WORKLOADS[args.workload]
    d = w.dynamics
    torch.cuda.init()
    r = time_workload(w, args.steps, args.warmup, args.observe_every, args.step_path,
                      args.autotune and not args.no_autotune)
    K = r["steps"]
    value = r["N"] * K / (r["ms"] * 1e-3)
    last = r["last"]
    line = {
        "metric": "LLG spin-updates/s at 1 GPU + HBM GB/s; surrogate vs direct dipole speedup at 1e-3",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "n_sites": r["N"], "lattice": w.description,
                   "alpha": d.alpha, "dt_ps": d.dt, "T_K": d.T, "observe_every": r["observe_every"],
                   "step_path": r["path"]},
        "hbm_gbps_algorithmic": value * BYTES_PER_UPDATE[w.precision] / 1e9,
        "roofline": roofline_of(w, r),
        "wall_s": r["wall_s"],
        "final_observation": {"E_per_spin": last["E"] / r["N"], "max_norm_dev": last["max_norm_dev"]},
    }
    extras = not args.no_extras
    if extras:
        line["config1"] = bench_config1(args)
    if extras or args.batch:
        line["batch"] = bench_batch(args)
    if extras or args.stencil:
        line["stencil"] = bench_stencil(args)
    if extras or args.basis:
        line["basis"] = bench_basis(args)
    if extras or args.surrogate:
        line["dipole"] = bench_surrogate(args)
    if args.tc:
        line["tc"] = bench_tc(args)
    pk.close_all()
    torch.cuda.synchronize()
    print("[bench] every engine, batch and chain closed", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
