"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

Workload (the paper's Table 2 size (32x2048)^2): L = 65536, 2^32 spins at
1 bit/spin (512 MiB per lattice), J = 1, beta in {0.40, 0.4406868, 0.50}, one
lattice per beta from the seed-7 start.  One step = one full sweep (black then
white half-sweep) of each of the three lattices; the default 200 steps are the
workload's 200 sweeps per beta.  The timed region starts from freshly
initialised lattices already resident in HBM.

Prints one JSON line: spin flips/ns (attempted single-spin updates per ns),
the half-sweep kernel against the HBM roofline (algorithmic bytes: target
read + write and source read, 3 bits per spin update), and the CPU oracle
timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
MFMA_FP16_PEAK_TFLOPS = 2500.0  # MI355X dense fp16 MFMA, TFLOP/s
# vector ALU: 256 compute units x 64 lanes x 2.4 GHz, one 32-bit lane operation
# per lane per cycle (a wave64 instruction takes 4 cycles on a 16-lane SIMD)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Philox4x32-10 blocks a 64-spin word takes on average near T_c under the lazy
# compare (host emulation of the kernels' decision on equilibrated lattices);
# with the generator's measured rate (philox_rate()) the rate no sweep that
# draws its random bits this way can exceed.
BLOCKS_PER_WORD = 3.84
KERNEL_SOURCES = ("paper_1906_06297_amd/csrc/sweep_kernels.hip",
                  "paper_1906_06297_amd/csrc/ising_device.hpp",
                  "paper_1906_06297_amd/csrc/ising_rows.hpp")
COUNTERS_SUMMARY = "profiles/half_sweep_L65536_counters.md"
N_SIMD = 1024  # 256 CUs x 4 SIMDs, one wave64 VALU instruction per 4 cycles each


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_summary() -> dict:
    """Values of the committed counter summary of the half-sweep, if it was taken
    on the kernel sources as they are now (else empty)."""
    path = os.path.join(ROOT, COUNTERS_SUMMARY)
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith(("source-sha256", "fetch_bytes_per_launch",
                                                        "write_bytes_per_launch",
                                                        "valu_insts_per_launch",
                                                        "shader_clock_ghz")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source-sha256") != kernel_source_hash():
        return {}
    return vals


def measured_traffic():
    """HBM bytes per half-sweep launch from the counter summary, or None."""
    vals = counter_summary()
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def valu_issue(avg_launch_us: float):
    """The vector-ALU side of the half-sweep: its wave-level VALU instructions
    per launch (counter summary) at one instruction per 4 cycles on each of the
    1024 SIMDs, against the measured launch time."""
    vals = counter_summary()
    try:
        insts, ghz = float(vals["valu_insts_per_launch"]), float(vals["shader_clock_ghz"])
    except (KeyError, ValueError):
        return None
    issue_us = insts * 4 / N_SIMD / (ghz * 1e3)
    return {"valu_insts_per_launch": insts, "shader_clock_ghz": ghz,
            "issue_us": issue_us, "frac_of_launch": issue_us / avg_launch_us}


def philox_rate(ising, torch) -> dict:
    """Philox4x32-10 blocks per second on the whole chip with the half-sweep's
    counter layout (ising_philox_rate: the generator alone), and the sweep
    rate it allows at BLOCKS_PER_WORD blocks per 64-spin word."""
    import ctypes

    from paper_1906_06297_amd import _lib

    nwords, nq = 1 << 25, 4  # the words of one half-sweep at L = 65536, 4 blocks each
    sink = torch.empty(256 * 2048, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def run():
        _lib.check(_lib.load().ising_philox_rate(nwords, nq, 7, 0, 1, ctypes.c_void_p(sink.data_ptr()),
                                                 sink.numel(), ctypes.c_void_p(stream)))

    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    rate = nwords * nq / sec
    return {"blocks_per_s": rate, "blocks_per_word": BLOCKS_PER_WORD,
            "ceiling_flips_per_ns": rate * 64 / BLOCKS_PER_WORD / 1e9,
            "probe": f"{nwords} words x {nq} blocks, {sec * 1e3:.3f} ms per launch"}


def onsager_energy(beta: float) -> float:
    """Infinite-lattice energy per site (Onsager 1944), J = 1, for reporting."""
    from scipy.special import ellipk

    K = beta
    kappa = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    m = min(kappa * kappa, 1.0)
    term = 0.0 if m >= 1.0 else (2 * math.tanh(2 * K) ** 2 - 1) * float(ellipk(m))
    return -1.0 / math.tanh(2 * K) * (1 + (2 / math.pi) * term)


def cpu_baseline(target_s: float = 15.0) -> dict:
    """The CPU oracle, as it stands, on a bounded sample of the workload."""
    import oracle

    oracle.lib()
    cores = oracle.max_threads()
    L, beta, seed = 8192, workloads.BETA_CRIT_CONFIG, workloads.HEADLINE["seed"]
    s = oracle.init(L, seed, 0)
    t0 = time.perf_counter()
    oracle.sweeps(s, beta, 1.0, seed, 0, 1, 0)
    one = time.perf_counter() - t0
    extra = max(0, min(1000, int(target_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    if extra:
        oracle.sweeps(s, beta, 1.0, seed, 0, extra, 1)
    dt = time.perf_counter() - t0
    nsw, secs = (extra, dt) if extra else (1, one)
    # one thread, a shorter sample of the same sweep
    oracle.set_threads(1)
    L1 = 2048
    s1 = oracle.init(L1, seed, 0)
    t0 = time.perf_counter()
    n1 = 0
    while time.perf_counter() - t0 < 3.0:
        oracle.sweeps(s1, beta, 1.0, seed, 0, 1, n1)
        n1 += 1
    single = n1 * L1 * L1 / ((time.perf_counter() - t0) * 1e9)
    oracle.set_threads(cores)
    return {
        "value": nsw * L * L / (secs * 1e9),
        "unit": "flips/ns",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"C/OpenMP int8 oracle (all 32 bit-planes per spin), {nsw} sweeps of an "
                   f"L={L} lattice at beta={beta} from the seed-{seed} start, {secs:.1f} s; "
                   f"one thread: {n1} sweeps of L={L1}"),
        "single_thread_value": single,
        "host_cpu": host_cpu(),
    }


def cpu_plan(ising, torch, progress) -> dict:
    """The oracle at the planned CPU-baseline sizes, each against the GPU on the
    same start: L = 64 (the correctness workload, 1000 sweeps at beta_c), L =
    4096 (200 sweeps per headline beta; the single-thread rate on the first 10
    sweeps per beta) and the first 4 sweeps of the headline lattice at beta_c;
    flips/ns on one thread and on all, and whether the lattices are
    identical."""
    import oracle

    oracle.lib()
    cores = oracle.max_threads()
    res = {"cores": cores, "host_cpu": host_cpu()}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    def gpu_spins(L, seed, stream, beta, n):
        lat = ising.Lattice(L, seed, stream)
        lat.sweep(beta, 1.0, n, 0)
        torch.cuda.synchronize()
        out = lat.get_spins()
        del lat
        return out

    c1 = workloads.CORRECTNESS
    L, n, beta = c1["L"], c1["nsweeps"], c1["beta"]
    row = {}
    for threads in (1, cores):
        oracle.set_threads(threads)
        s = oracle.init(L, c1["seed"], c1["stream"])
        dt = timed(lambda: oracle.sweeps(s, beta, 1.0, c1["seed"], c1["stream"], n, 0))
        row[f"flips_per_ns_{threads}_threads"] = n * L * L / (dt * 1e9)
    row["bit_exact"] = bool(np.array_equal(s, gpu_spins(L, c1["seed"], c1["stream"], beta, n)))
    res[f"L{L}_{n}_sweeps"] = row
    progress("CPU plan: L = 64 done")

    L, n = 4096, 200
    row = {"betas": list(workloads.HEADLINE["betas"])}
    oracle.set_threads(cores)
    secs, ok = 0.0, True
    for beta in workloads.HEADLINE["betas"]:
        s = oracle.init(L, workloads.HEADLINE["seed"], 0)
        secs += timed(lambda: oracle.sweeps(s, beta, 1.0, workloads.HEADLINE["seed"], 0, n, 0))
        ok = ok and bool(np.array_equal(s, gpu_spins(L, workloads.HEADLINE["seed"], 0, beta, n)))
    row[f"flips_per_ns_{cores}_threads"] = 3 * n * L * L / (secs * 1e9)
    row["wall_s_all_threads"] = secs
    row["bit_exact"] = ok
    oracle.set_threads(1)
    n1, secs1 = 10, 0.0
    for beta in workloads.HEADLINE["betas"]:
        s = oracle.init(L, workloads.HEADLINE["seed"], 0)
        secs1 += timed(lambda: oracle.sweeps(s, beta, 1.0, workloads.HEADLINE["seed"], 0, n1, 0))
    row["flips_per_ns_1_threads"] = 3 * n1 * L * L / (secs1 * 1e9)
    row["single_thread_sample"] = f"first {n1} sweeps per beta"
    res[f"L{L}_{n}_sweeps"] = row
    oracle.set_threads(cores)
    progress("CPU plan: L = 4096 done")

    cfg = workloads.HEADLINE
    L, n, beta = cfg["L"], 4, workloads.BETA_CRIT_CONFIG
    s = oracle.init(L, cfg["seed"], cfg["stream"])
    secs = timed(lambda: oracle.sweeps(s, beta, 1.0, cfg["seed"], cfg["stream"], n, 0))
    ok = bool(np.array_equal(s, gpu_spins(L, cfg["seed"], cfg["stream"], beta, n)))
    del s
    res[f"L{L}_first_{n}_sweeps"] = {"beta": beta, "wall_s": secs,
                                     f"flips_per_ns_{cores}_threads": n * L * L / (secs * 1e9),
                                     "bit_exact": ok}
    progress("CPU plan: L = 65536 done")
    return res


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batched(ising, torch, nsweeps: int, philox_ceiling: float) -> dict:
    """The batched workload: 1024 lattices of uneven L and beta in one persistent launch."""
    cfg = workloads.BATCHED
    Ls, betas, seeds, streams = workloads.batched_lattices()
    b = ising.Batch(Ls, betas, cfg["J"], seeds, streams)
    t0 = time.perf_counter()
    tiles = b.autotune(200, None)
    tune_s = time.perf_counter() - t0
    plans = {L: b.plan(L) for L in tiles}
    mixed = b.mixed()
    b.init()
    b.sweep(nsweeps)  # captures the graph (untimed), then a timed replay from a fresh start
    b.init()
    b.set_counter(0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.sweep(nsweeps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    updates = float(sum(int(L) * int(L) for L in Ls)) * nsweeps
    # the largest lattices alone bound the makespan of one launch
    big = [q for q in range(len(Ls)) if Ls[q] == max(Ls)]
    bb = ising.Batch([Ls[q] for q in big], [betas[q] for q in big], cfg["J"],
                     [seeds[q] for q in big], [streams[q] for q in big])
    bb.autotune(200, None)  # the largest size tuned on its own: a bound on the makespan
    bb.init()
    bb.sweep(nsweeps)
    bb.init()
    bb.set_counter(0)
    torch.cuda.synchronize()
    e0.record()
    bb.sweep(nsweeps)
    e1.record()
    torch.cuda.synchronize()
    big_ms = e0.elapsed_time(e1)
    b.close()
    bb.close()
    return {
        "workload": "1024 lattices, L uniform over {16,...,256}, beta over linspace(0.30,0.60,32), "
                    f"{nsweeps} sweeps each, one graph-replayed persistent launch",
        "flips_per_ns": updates / (ms * 1e6),
        "ms": ms,
        "updates": updates,
        "largest_size_alone_ms": big_ms,
        "largest_size_count": len(big),
        "tiles_words_lanes": {str(k): list(v) for k, v in tiles.items()},
        "lattices_per_workgroup_and_workgroups": {str(k): list(plans[k]) for k in plans},
        "mixed_size_workgroups": mixed,
        "autotune_s": tune_s,
        "philox_ceiling_flips_per_ns": philox_ceiling,
        "frac_of_philox_ceiling": updates / (ms * 1e6) / philox_ceiling,
    }


def bench_heatbath(ising, torch, bufs, steps: int) -> dict:
    """The headline workload under the heat-bath rule (Sec. 2): same lattices,
    betas and start; every class draws random numbers."""
    cfg = workloads.HEADLINE
    L, betas, seed, J = cfg["L"], cfg["betas"], cfg["seed"], cfg["J"]
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    for lat, beta in zip(lats, betas):
        lat.sweep(beta, J, 1, 0, rule="heatbath")
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    torch.cuda.synchronize()
    per_beta = {}
    t_all = 0.0
    for lat, beta in zip(lats, betas):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lat.sweep(beta, J, steps, 0, rule="heatbath")
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        t_all += ms
        bond, mag = lat.observables()
        per_beta[str(beta)] = {"flips_per_ns": steps * L * L / (ms * 1e6),
                               "E_per_site": -J * bond / (L * L),
                               "onsager_E_per_site": onsager_energy(beta * J)}
    half_us = t_all * 1e3 / (2 * steps * len(betas))
    return {
        "workload": f"heat-bath checkerboard sweeps, L={L}, J={J}, beta in {list(betas)}, seed {seed}, "
                    f"{steps} sweeps per beta from a fresh start",
        "flips_per_ns": len(betas) * steps * L * L / (t_all * 1e6),
        "avg_half_sweep_us": half_us,
        "hbm_frac": 805306368 / (half_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "per_beta": per_beta,
    }


def bench_glass(ising, torch, bufs, steps: int) -> dict:
    """+-J spin glass on the headline lattices: random bond signs (probability
    1/2, their own Philox key), same spins, betas and start as the headline."""
    cfg = workloads.GLASS
    L, betas, seed, J = cfg["L"], cfg["betas"], cfg["seed"], cfg["J"]
    bonds = ising.GlassBonds(L, seed=cfg["coupling_seed"], stream_id=0)
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    for lat, beta in zip(lats, betas):
        lat.glass_sweep(bonds, beta, J, 1, 0)
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    torch.cuda.synchronize()
    per_beta, t_all = {}, 0.0
    for lat, beta in zip(lats, betas):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lat.glass_sweep(bonds, beta, J, steps, 0)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        t_all += ms
        bond, _ = lat.glass_observables(bonds)
        per_beta[str(beta)] = {"flips_per_ns": steps * L * L / (ms * 1e6),
                               "E_per_site": -J * bond / (L * L)}
    half_us = t_all * 1e3 / (2 * steps * len(betas))
    alg = 7 * (L * L // 2) // 8  # target read + write, source read, four bond bits per update
    del bonds
    return {
        "workload": f"+-J spin glass, L={L}, J={J}, bond signs -1 with probability 1/2 (Philox "
                    f"domain 4, seed {cfg['coupling_seed']}), beta in {list(betas)}, spins seed {seed}, "
                    f"{steps} sweeps per beta from a fresh start",
        "flips_per_ns": len(betas) * steps * L * L / (t_all * 1e6),
        "avg_half_sweep_us": half_us,
        "alg_bytes_per_launch": alg,
        "hbm_frac": alg / (half_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "per_beta": per_beta,
    }


def bench_matmul(ising, torch, steps: int, sizes=None) -> dict:
    """The matrix-multiply formulation of the sweep (Sec. 3.2, the tensor-core
    implementation) against the bit-packed kernel on the same lattices: the
    paper's tensor-core lattice sizes (20..640 x 128)^2 and the headline
    L = 65536, beta_c, seed 7, from a fresh start each.  Both matmul forms
    yield the bit-packed kernel's lattice bit for bit."""
    beta, J, seed = workloads.BETA_CRIT_CONFIG, 1.0, 7
    if not sizes:
        sizes = [128 * f for f in (20, 40, 80, 160, 320, 640)] + [65536]
    rows = []
    head = None
    for L in sizes:
        n = max(steps, min(200, int(5e9 / (L * L))))
        row = {"L": L, "sweeps": n}

        def timed(fn):
            fn(1, 0)  # warmup sweep
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(n, 1)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n  # ms per sweep

        lat = ising.Lattice(L, seed)
        ms = timed(lambda k, ctr: lat.sweep(beta, J, k, ctr))
        row["bitpacked_flips_per_ns"] = L * L / (ms * 1e6)
        for fused, key in ((True, "mm_fused"), (False, "mm_three_kernel")):
            lat = ising.Lattice(L, seed)
            mm = ising.MatmulLattice(lat, fused=fused)
            ms = timed(lambda k, ctr: mm.sweep(beta, J, k, ctr))
            row[f"{key}_flips_per_ns"] = L * L / (ms * 1e6)
            row[f"{key}_half_sweep_us"] = ms * 1e3 / 2
            del mm
            torch.cuda.empty_cache()
        del lat
        torch.cuda.empty_cache()
        row["bitpacked_over_mm_fused"] = row["bitpacked_flips_per_ns"] / row["mm_fused_flips_per_ns"]
        rows.append(row)
        if L == 65536:
            head = row
    out = {
        "workload": f"matrix-multiply neighbour sums (fp16 MFMA 16x16x32, 128 x 128 blocks of "
                    f"256 x 256 sub-lattices) vs the bit-packed kernel, beta {beta}, J {J}, seed "
                    f"{seed}, L in {sizes}",
        "per_L": rows,
    }
    if head is not None:
        # the fused kernel at L = 65536: dense fp16 MFMA work and the bytes an
        # fp16 half-sweep must move (source colour read, target read and written)
        tiles = 2 * (65536 // 256) ** 2
        flops = tiles * 2 * 2 * 128 ** 3
        byts = 6 * (65536 * 65536 // 2)
        us = head["mm_fused_half_sweep_us"]
        out["fused_L65536"] = {
            "mfma_dense_tflops": flops / (us * 1e-6) / 1e12,
            "mfma_frac_of_fp16_peak": flops / (us * 1e-6) / 1e12 / MFMA_FP16_PEAK_TFLOPS,
            "useful_flop_fraction": 1 / 64,
            "alg_bytes_per_launch": byts,
            "hbm_frac": byts / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        }
    return out


def bench_hybrid64(ising, torch, sweeps: int, data_log2: int = 20, train_steps: int = 2000,
                   batch: int = 128) -> dict:
    """The hybrid chain at L = 64: 16 betas in [0.40, 0.48] with 16 chains each,
    a 64-channel network trained on 2^data_log2 plain-sampler configurations
    pooled over those betas, one global move per 10 local sweeps, against
    independent plain chains: E per site and Binder cumulant with jackknife
    errors, tau_int(|m|) per measurement, acceptance, and effective samples
    per second."""
    from paper_1906_06297_amd import hybrid

    L, C = 64, 64
    betas = np.linspace(0.40, 0.48, 16)
    chains_data = 4096
    t0 = time.perf_counter()
    data = hybrid.plain_configurations(L, betas, chains=chains_data,
                                       snapshots=(1 << data_log2) // chains_data, thin=10,
                                       burn=20000, seed=61, stream_base=4096)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = ising.ARNet(L, C, 256)
    try:
        net.set_params(hybrid.init_params(L, C, seed=3))
        t0 = time.perf_counter()
        hist = hybrid.train(net, data, steps=train_steps, batch=batch, lr=2e-3, seed=4,
                            log_every=max(1, train_steps // 5))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del data
        res = hybrid.compare_over_betas(net, L, betas, per_beta=16, sweeps=sweeps,
                                        sweeps_per_proposal=10, burn=20000, seed_plain=71,
                                        seed_hybrid=72)
    finally:
        net.close()
    out = {"per_beta": [], "data_s": t_data, "train_s": t_train, "train_nll_per_site": hist}
    z = []
    for p, h in zip(res["plain"]["per_beta"], res["hybrid"]["per_beta"]):
        row = {"beta": p["beta"]}
        for kind, r in (("plain", p), ("hybrid", h)):
            row[kind] = {k: r[k] for k in ("E_per_site", "E_se", "binder", "binder_se",
                                           "tau_int_abs_m", "acceptance")}
        row["z_E"] = (h["E_per_site"] - p["E_per_site"]) / float(np.hypot(p["E_se"], h["E_se"]))
        row["z_binder"] = (h["binder"] - p["binder"]) / float(np.hypot(p["binder_se"], h["binder_se"]))
        z += [row["z_E"], row["z_binder"]]
        row["learned_vs_plain"] = ("measured" if h["acceptance"] > 0 else
                                   "unmeasured: no proposal accepted, the hybrid chain is the plain "
                                   "chain at this beta")
        out["per_beta"].append(row)
    n_meas = res["plain"]["measurements"] * 16  # measurements x chains, per beta
    for kind in ("plain", "hybrid"):
        taus = np.array([r["tau_int_abs_m"] for r in res[kind]["per_beta"]])
        out[f"{kind}_wall_s"] = res[kind]["wall_s"]
        out[f"{kind}_ess_per_s_abs_m"] = float(np.sum(n_meas / (2 * taus)) / res[kind]["wall_s"])
    out["max_abs_z"] = float(np.max(np.abs(z)))
    out["betas_with_accepted_proposals"] = int(sum(r["hybrid"]["acceptance"] > 0
                                                   for r in out["per_beta"]))
    out["workload"] = (f"L={L}, 16 betas in [0.40, 0.48] x 16 chains, {C}-channel net trained "
                       f"{train_steps} Adam steps (batch {batch}) on 2^{data_log2} plain-sampler "
                       f"configurations pooled over the betas; {sweeps} sweeps after 20000 burn-in, a "
                       "global move every 10 sweeps (hybrid) against independent plain chains")
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 MFMA, TFLOP/s


def bench_learned_kernels(ising, torch) -> dict:
    """The learned proposal's kernels at the workload shapes (L = 32, 32
    channels, 4096 proposals, training batch 256; L = 64, 64 channels, 256
    proposals, training batch 64), random bf16 weights: ms per call of the
    sampler (anti-diagonal, one configuration per workgroup), the evaluator
    (log q~ of a batch) and one training step (forward, backward, Adam), with
    the MFMA work of layers 2..6 (2 flops per multiply-add of 5C x C per site and
    layer, 5C for layer 6) against the bf16 MFMA peak."""
    from paper_1906_06297_amd import hybrid

    def timeit(fn, n=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {}
    for L, C, B, Bt in ((32, 32, 4096, 256), (64, 64, 256, 64)):
        net = ising.ARNet(L, C, B)
        try:
            net.set_params(hybrid.init_params(L, C, seed=5))
            x, _ = net.sample(B, seed=1)
            xb = x[:Bt].contiguous()
            ms = {"sample": timeit(lambda: net.sample(B, seed=1, round=2)),
                  "log_prob": timeit(lambda: net.log_prob(x)),
                  "train_step": timeit(lambda: net.train_step(xb, 1e-5))}
        finally:
            net.close()
        flops_site = 2 * (4 * 5 * C * C + 5 * C)
        work = {"sample": flops_site * L * L * B, "log_prob": flops_site * L * L * B,
                "train_step": 3 * flops_site * L * L * Bt}  # forward, data and weight gradients
        out[f"L{L}_C{C}"] = {
            "batch": B, "train_batch": Bt, "ms": ms,
            "mfma_tflops": {k: work[k] / (ms[k] * 1e-3) / 1e12 for k in ms},
            "frac_of_bf16_mfma_peak": {k: work[k] / (ms[k] * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS
                                       for k in ms},
        }
    return out


def bench_learned(ising, torch, L: int = 32, betas=(0.42, 0.44, 0.46), C: int = 32,
                  chains: int = 4096, rounds: int = 400, train_steps: int = 4000,
                  data_log2: int = 20) -> dict:
    """Learned global proposal against the plain sweep on the same GPU, per beta:
    a network trained on 2^data_log2 plain-sampler configurations at that beta,
    then `chains` chains per kind; per round one local sweep, plus one proposal
    in the hybrid chains (a batch of `chains` proposals).  tau_int of |m| and E
    per round, effective samples per second, and the observables of both."""
    from paper_1906_06297_amd import hybrid, stats

    snapshots = (1 << data_log2) // chains
    out = {}
    for bi, beta in enumerate(betas):
        t0 = time.perf_counter()
        data = hybrid.plain_configurations(L, beta, chains=chains, snapshots=snapshots, thin=10,
                                           burn=1000, seed=41 + bi, stream_base=1 << 20)
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        net = ising.ARNet(L, C, chains)
        net.set_params(hybrid.init_params(L, C, seed=1))
        t0 = time.perf_counter()
        hist = hybrid.train(net, data, steps=train_steps, batch=256, lr=2e-3, seed=2 + bi,
                            log_every=max(1, train_steps // 5))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del data
        res = {}
        for name, use in (("plain", None), ("hybrid", net)):
            ch = hybrid.Chains(L, [beta] * chains, seed=43 + bi, stream_base=0)
            ch.local(1000)  # burn-in by plain sweeps, the same for both kinds
            E, A, wall, accepted = hybrid.run_series(ch, rounds, 1, use, seed=47 + bi,
                                                     round0=10_000)
            acc = float(accepted.sum()) / (chains * rounds) if accepted is not None else None
            ch.close()
            tau_m, tau_e = stats.tau_int_chains(A), stats.tau_int_chains(E)
            pe, pm = E.mean(axis=0), A.mean(axis=0)
            res[name] = {
                "acceptance": acc,
                "tau_int_abs_m_rounds": tau_m,
                "tau_int_E_rounds": tau_e,
                "ms_per_round": wall / rounds * 1e3,
                "ess_per_s_abs_m": chains * rounds / (2 * tau_m) / wall,
                "ess_per_s_E": chains * rounds / (2 * tau_e) / wall,
                "E_per_site": float(pe.mean()), "E_se": float(pe.std(ddof=1) / np.sqrt(chains)),
                "abs_m": float(pm.mean()), "abs_m_se": float(pm.std(ddof=1) / np.sqrt(chains)),
            }
        net.close()
        # wall time the hybrid chains need for the standard error the plain chains reach
        # in the same wall time, relative to the plain chains (ESS/s ratio)
        res["hybrid_wall_for_matched_error"] = {
            obs: res["plain"][f"ess_per_s_{obs}"] / res["hybrid"][f"ess_per_s_{obs}"]
            for obs in ("abs_m", "E")}
        out[str(beta)] = {"train_nll_per_site": hist, "data_s": t_data, "train_s": t_train, **res}
    return {
        "workload": f"L={L}, beta in {list(betas)}: per beta a {C}-channel masked-conv "
                    f"autoregressive proposal (6 layers, bf16 weights, fp32 sums) trained on 2^{data_log2} "
                    f"plain-sampler configurations ({train_steps} Adam steps, batch 256, flip/translation "
                    f"augmentation); {chains} chains x {rounds} rounds after 1000 plain burn-in sweeps, "
                    f"a round = 1 sweep (+ 1 proposal per chain in hybrid, MH accept in fp32)",
        "per_beta": out,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=workloads.HEADLINE["nsweeps"])
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle timing (for profiler runs)")
    ap.add_argument("--batched-sweeps", type=int, default=workloads.BATCHED["nsweeps"],
                    help="sweeps of the batched workload reported beside the headline (0 = skip)")
    ap.add_argument("--learned-rounds", type=int, default=400,
                    help="rounds of the learned-proposal comparison reported beside the headline "
                         "(0 = skip)")
    ap.add_argument("--heatbath-sweeps", type=int, default=20,
                    help="sweeps per beta of the heat-bath rule on the headline lattices, reported "
                         "beside the headline (0 = skip)")
    ap.add_argument("--glass-sweeps", type=int, default=20,
                    help="sweeps per beta of the +-J spin glass on the headline lattices (0 = skip)")
    ap.add_argument("--learned-kernels", type=int, default=1,
                    help="time the learned proposal's kernels at the workload shapes (0 = skip)")
    ap.add_argument("--hybrid64-sweeps", type=int, default=100000,
                    help="sweeps of the L = 64 hybrid-chain comparison (0 = skip)")
    ap.add_argument("--matmul-sweeps", type=int, default=5,
                    help="minimum sweeps per size of the matrix-multiply comparison (0 = skip)")
    ap.add_argument("--matmul-L", type=int, nargs="*", default=None,
                    help="lattice sizes of the matrix-multiply comparison (default: the paper's "
                         "tensor-core sizes and 65536)")
    ap.add_argument("--hold-seconds", type=float, default=0.0,
                    help="only run L = 65536 sweeps at beta_c for this many seconds (for reading "
                         "clocks and power beside a steady load) and exit")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the hash of the half-sweep kernel sources and exit")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="also time the oracle at the planned CPU-baseline sizes (L = 64, 4096 and "
                         "the first 4 headline sweeps), each checked against the GPU")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three plain 1 GiB device-to-device copies, whose HBM counter "
                         "readings scale the profiler's byte counts")
    args = ap.parse_args()
    t_start = time.perf_counter()
    if args.print_source_hash:
        print(kernel_source_hash())
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sweep is "
              "built and measured on a single MI355X)", file=sys.stderr)
        return 2

    import torch

    import paper_1906_06297_amd as ising

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.hold_seconds > 0:
        lat = ising.Lattice(workloads.HEADLINE["L"], workloads.HEADLINE["seed"])
        t0, n = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.hold_seconds:
            lat.sweep(workloads.BETA_CRIT_CONFIG, 1.0, 50, n)
            torch.cuda.synchronize()
            n += 50
        print(f"held: {n} sweeps, {(time.perf_counter() - t0) / (2 * n) * 1e6:.1f} us per "
              "half-sweep", flush=True)
        return 0
    cfg = workloads.HEADLINE
    L, betas, seed, J = cfg["L"], cfg["betas"], cfg["seed"], cfg["J"]
    K, Wm = args.steps, args.warmup
    W = ising.words_per_colour(L)
    bufs = [torch.empty(2 * W, dtype=torch.int64, device="cuda") for _ in betas]

    # warmup on the same buffers, then a fresh start for the timed region
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    for lat, beta in zip(lats, betas):
        lat.sweep(beta, J, Wm, 0)
    lats = [ising.Lattice(L, seed, words=b) for b in bufs]
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in betas]
    t0 = time.perf_counter()
    for (e0, e1), lat, beta in zip(ev, lats, betas):
        e0.record()
        lat.sweep(beta, J, K, 0)
        e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_beta_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    gpu_ms = sum(per_beta_ms)

    updates = len(betas) * K * L * L
    value = updates / (wall * 1e9)
    half_sweep_ms = gpu_ms / (len(betas) * 2 * K)
    alg_bytes = 3 * (L * L // 2) // 8  # target read + write, source read: 3 bits per update
    achieved = alg_bytes / (half_sweep_ms * 1e-3) / 1e9

    philox = philox_rate(ising, torch)
    valu = valu_issue(half_sweep_ms * 1e3)
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes}
    if valu is not None:
        # the binding limit: vector-ALU issue (instructions per launch from the
        # counter summary, at 64 lane operations each, over the live launch time)
        lane_tops = valu["valu_insts_per_launch"] * 64 / (half_sweep_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": lane_tops, "peak": VALU_PEAK_TOPS,
                    "unit": "Tops/s (32-bit VALU lane operations)", "frac": lane_tops / VALU_PEAK_TOPS}
    else:  # counters not taken on these sources: the HBM roof only
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS}
    roofline.update({
        "kernel": "half-sweep",
        "traffic": measured_traffic(),
        "avg_launch_us": half_sweep_ms * 1e3,
        "hbm": hbm,
        "valu": valu,
        "philox": philox,
        "frac_of_philox_ceiling": (L * L / 2) / (half_sweep_ms * 1e6) / philox["ceiling_flips_per_ns"],
    })

    physics = {}
    for lat, beta, ms in zip(lats, betas, per_beta_ms):
        bond, mag = lat.observables()
        physics[f"{beta}"] = {
            "flips_per_ns": K * L * L / (ms * 1e6),
            "E_per_site": -J * bond / (L * L),
            "onsager_E_per_site": onsager_energy(beta),
            "abs_m": abs(mag) / (L * L),
        }

    out = {
        "metric": "spin flips/ns + % HBM roofline (1 GPU)",
        "value": value,
        "unit": "flips/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 (1 bit/spin), u32 Philox",
        "data": "synthetic",
        "config": {
            "workload": "checkerboard Metropolis, L=65536 (2^32 spins, 512 MiB at 1 bit/spin), "
                        "J=1, beta in {0.40, 0.4406868, 0.50}, seed 7, one full sweep per beta "
                        "per step from a fresh start",
            "L": L,
            "betas": list(betas),
            "sweeps_per_beta": K,
            "per_beta": physics,
        },
        "roofline": roofline,
    }
    def progress(msg):  # stderr: the JSON line stays the only thing on stdout
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    progress(f"headline: {value:.0f} flips/ns")
    if args.heatbath_sweeps > 0:
        out["heatbath"] = bench_heatbath(ising, torch, bufs, args.heatbath_sweeps)
        progress("heat bath done")
    if args.glass_sweeps > 0:
        out["glass"] = bench_glass(ising, torch, bufs, args.glass_sweeps)
        progress("spin glass done")
    if args.matmul_sweeps > 0:
        out["matmul"] = bench_matmul(ising, torch, args.matmul_sweeps, args.matmul_L)
        progress("matrix-multiply comparison done")
    if args.batched_sweeps > 0:
        out["batched"] = bench_batched(ising, torch, args.batched_sweeps,
                                       philox["ceiling_flips_per_ns"])
        progress("batched done")
    if args.learned_kernels > 0:
        out["learned_kernels"] = bench_learned_kernels(ising, torch)
        progress("learned kernels done")
    if args.learned_rounds > 0:
        out["learned"] = bench_learned(ising, torch, rounds=args.learned_rounds)
        progress("learned proposal at L = 32 done")
    if args.hybrid64_sweeps > 0:
        out["hybrid_L64"] = bench_hybrid64(ising, torch, args.hybrid64_sweeps)
        progress("hybrid chains at L = 64 done")
    if args.copy_calibration:
        del bufs, lats
        a = torch.empty(1 << 27, dtype=torch.int64, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 8
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        progress("CPU baseline done")
    if args.cpu_plan:
        out["cpu_plan"] = cpu_plan(ising, torch, progress)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
