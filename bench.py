"""Benchmark: log marginal likelihood + gradient of a Matern-5/2 GP at N = 2^20 in FP64.

One step = one spingp_logml_grad call on resident synthetic input (bound and validated once by
spingp_assemble, as in a training loop whose optimiser updates the hyperparameters in device
memory): chunk fold and work-group trees, top-level tree and down-sweeps, chunk elimination +
adjoint sweep + gradient sum.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Arithmetic per point of the two per-point kernels, counted from their formulas (FMA = 2 flops,
# a divide, exp or log = 1), b = 3.  The O(N/R) work-group and top-level trees are parallel
# overhead and are not counted as algorithmic work.
FLOPS_PER_POINT = {
    "fwd_fold_tree": 259.0,     # rank-one fold of one node into the chunk element
    "bwd_elim_adjoint": 542.0,  # Kalman elimination step (170) + adjoint step (372)
}
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0
MACHINE_BALANCE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)   # flop per HBM byte, 9.8
# Algorithmic HBM bytes per point of the two per-point kernels: t and y read once each.
ALG_BYTES_PER_POINT = {"fwd_fold_tree": 16.0, "bwd_elim_adjoint": 16.0}

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes on
# this workload, per tile shape (R, L), scaled by a 256 MiB copy (FETCH x 2.0, WRITE x 1.0);
# valid only for the kernel sources they were taken on (sha256 over the one-series kernel
# sources, see kernel_source_sha), else reported as null.
TRAFFIC = {"kernel": "bwd_elim_adjoint",
           "bytes": {(8, 128): (40792.9 * 2.0 + 96.0) * 1024.0,
                     (8, 256): (38869.7 * 2.0 + 48.0) * 1024.0},
           "source_sha": "eff41554fdd90400e11f3a990899cf592f419c2be1e8231dbc1efea30763565b"}


def kernel_source_sha():
    """Hash of the sources the one-series Matern kernels are built from (the counters in TRAFFIC
    hold for exactly these)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1610_08035_amd", "csrc")
    h = hashlib.sha256()
    for f in ("spingp_device.hpp", "spingp_host.hpp", "spingp_kernels.hpp", "spingp_series.hpp",
              "spingp_tile.hip"):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def host_cpu():
    """CPU model and thread counts of the host this runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_config1(reps=5):
    """Config 1 on the host (Matern-3/2, N = 1000; posterior mean, variances, logML): median of
    `reps` runs of the C sequential elimination (one thread), the Python Kalman filter + RTS
    smoother (one thread) and, as context, the dense GP (numpy/LAPACK, the BLAS's threads)."""
    from oracle import dense, kalman, native
    from oracle.ssm import model_for
    from workloads import make_config
    w = make_config(1)
    t, y, hyp = w.series(0)
    m = model_for(w.terms, hyp)
    out = {}
    for name, fn in (("c_elimination", lambda: native.btd_factored(w.terms, hyp, t, y, want_blocks=False)),
                     ("python_kalman_rts", lambda: kalman.kf_rts(m, t, y)),
                     ("dense_gp", lambda: dense.gp_dense(m, t, y, want_grad=False))):
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t0)
        out[name] = {"seconds": float(np.median(times)), "points_per_s": t.shape[0] / float(np.median(times))}
    out["c_elimination"]["cores"] = 1
    out["python_kalman_rts"]["cores"] = 1
    out["dense_gp"]["cores"] = "BLAS threads"
    return {"workload": "matern32_n1000_uniform100_mean_var_logml", "n_points": int(t.shape[0]), "reps": reps,
            **out}


_W4 = None


def _workload4():
    """The 4096-series batch, generated once per process."""
    global _W4
    if _W4 is None:
        from workloads import make_config
        _W4 = make_config(4)
    return _W4


def _cpu_series_grad(args):
    """logML + gradient of a range of series of the 4096-series batch by the C oracle (one
    process; the batch is generated before the timed calls)."""
    from oracle import native
    lo, hi = args
    w = _workload4()
    for i in range(lo, hi):
        t, y, hyp = w.series(i)
        native.tangent_grad(w.terms, hyp, t, y)
    return hi - lo


def _cpu_worker_ready(_):
    _workload4()
    time.sleep(0.2)
    return os.getpid()


def cpu_table():
    """The CPU oracle on every workload, on this host: C sequential elimination (one thread) for
    the forward outputs, C tangent-linear logML + gradient (one thread) for the gradient
    workloads, and for the 4096-series batch also all usable cores (series spread over worker
    processes).  Median of 3 runs where a run takes under 5 s, else one run."""
    import concurrent.futures
    from oracle import native
    from workloads import make_config

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        el = time.perf_counter() - t0
        if el < 5.0:
            runs = [el]
            for _ in range(2):
                t0 = time.perf_counter()
                fn()
                runs.append(time.perf_counter() - t0)
            el = float(np.median(runs))
        return el

    rows = {"host": host_cpu(), "config1": cpu_config1()}
    w = make_config(2)
    t, y, hyp = w.series(0)
    el = timed(lambda: native.btd_factored(w.terms, hyp, t, y, want_blocks=False))
    rows["config2_forward"] = {"what": "factor, logML, mean, variance (C elimination)", "cores": 1,
                               "n_points": int(t.shape[0]), "seconds": el, "points_per_s": t.shape[0] / el}
    print("cpu table: config2_forward done", file=sys.stderr, flush=True)
    el = timed(lambda: native.tangent_grad(w.terms, hyp, t, y))
    rows["headline_logml_grad"] = {"what": "logML + 3-parameter gradient (C tangent-linear)", "cores": 1,
                                   "n_points": int(t.shape[0]), "seconds": el, "points_per_s": t.shape[0] / el}
    print("cpu table: headline_logml_grad done", file=sys.stderr, flush=True)
    w3 = make_config(3)
    t3, y3, h3 = w3.series(0)
    el = timed(lambda: native.tangent_grad(w3.terms, h3, t3, y3))
    rows["config3_sum_kernel"] = {"what": "b = 10 logML + 6-parameter gradient (C tangent-linear)", "cores": 1,
                                  "n_points": int(t3.shape[0]), "seconds": el, "points_per_s": t3.shape[0] / el}
    print("cpu table: config3_sum_kernel done", file=sys.stderr, flush=True)
    w4 = _workload4()
    el1 = timed(lambda: _cpu_series_grad((0, w4.n_series)))
    cores = host_cpu()["usable_cpus"] or 1
    step = max(1, -(-w4.n_series // (4 * cores)))
    chunks = [(i, min(i + step, w4.n_series)) for i in range(0, w4.n_series, step)]
    with concurrent.futures.ProcessPoolExecutor(cores) as ex:
        # start every worker and let each generate the batch before the timed map
        ready = set(ex.map(_cpu_worker_ready, range(4 * cores)))
        t0 = time.perf_counter()
        list(ex.map(_cpu_series_grad, chunks))
        eln = time.perf_counter() - t0
    rows["config4_batched"] = {"what": "4096 series, logML + gradient each (C tangent-linear)",
                               "n_points": int(w4.n_points), "one_core": {"seconds": el1, "points_per_s": w4.n_points / el1},
                               "all_cores": {"cores": cores, "workers_started": len(ready), "seconds": eln,
                                             "points_per_s": w4.n_points / eln}}
    print("cpu table: config4_batched done", file=sys.stderr, flush=True)
    w5 = make_config(5)
    t5, y5, h5 = w5.series(0)
    el = timed(lambda: native.tangent_grad(w5.terms, h5, t5, y5))
    rows["config5_large"] = {"what": "N = 2^24 logML + gradient (C tangent-linear)", "cores": 1,
                             "n_points": int(t5.shape[0]), "seconds": el, "points_per_s": t5.shape[0] / el}
    print("cpu table: config5_large done", file=sys.stderr, flush=True)
    return rows


def cpu_baseline(w, budget_s=10.0):
    """The C oracle (sequential elimination + tangent-linear gradient), timed on the host.

    The sample is the whole series, repeated until about `budget_s` seconds of CPU work
    (a single pass over 2^20 points takes well under a second)."""
    from oracle import native
    t, y, hyp = w.series(0)
    reps, total, pts = 0, 0.0, 0
    while total < budget_s and reps < 1000:
        t0 = time.perf_counter()
        native.tangent_grad(w.terms, hyp, t, y)
        total += time.perf_counter() - t0
        pts += t.shape[0]
        reps += 1
    return {"value": pts / total, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"all {t.shape[0]} points x {reps} repetitions ({total:.1f} s): logML + 3-parameter "
                      f"gradient by the single-threaded C sequential elimination with tangent-linear derivatives",
            "host": host_cpu()}


def batched_report(spg, steps, warmup):
    """4096 independent Matern-5/2 series (lengths log-uniform in [64, 16384]) in one batched
    call (autotuned tile shape, eager launches on a side stream) against one single-series call
    per series on pre-assembled handles, same GPU, same stream, same inputs resident in device
    memory."""
    import torch
    from workloads import make_config
    w = make_config(4)
    dev = torch.device("cuda:0")
    td, yd = torch.as_tensor(w.t, device=dev), torch.as_tensor(w.y, device=dev)
    hd = torch.as_tensor(w.hyper.reshape(-1), device=dev)
    od = torch.as_tensor(w.offsets, device=dev)
    S, n = w.n_series, w.n_points
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    h = spg.Handle(w.terms, n, S, stream=side)
    h.assemble(td, yd, hd, od, autotune=True)
    ll = torch.empty(S, dtype=torch.float64, device=dev)
    g = torch.empty(S, 3, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    if h.status()[0] != 0:
        raise RuntimeError("batched workload failed validation")
    t0 = time.perf_counter()
    for _ in range(steps):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    el_b = (time.perf_counter() - t0) / steps
    R, L = spg.spingp_tile_shape(h.tile)
    # the same steps as replays of the captured launch sequence (same tile, same stream)
    hg = spg.Handle(w.terms, n, S, stream=side)
    hg.tile = h.tile
    hg.assemble(td, yd, hd, od, graph=True)
    for _ in range(warmup):
        spg.spingp_logml_grad(hg._h, ll, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        spg.spingp_logml_grad(hg._h, ll, g)
    torch.cuda.synchronize()
    el_g = (time.perf_counter() - t0) / steps
    hg.close()
    h.close()
    # one handle and one call per series
    hs, outs = [], []
    for s in range(S):
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        hh = spg.Handle(w.terms, e - a, stream=side)
        hh.assemble(td[a:e], yd[a:e], hd[3 * s: 3 * s + 3])
        hs.append(hh)
        outs.append((ll[s: s + 1], g[s: s + 1]))
    for _ in range(max(1, warmup // 2)):
        for hh, (l1, g1) in zip(hs, outs):
            spg.spingp_logml_grad(hh._h, l1, g1)
    torch.cuda.synchronize()
    ps_steps = max(1, min(10, steps // 4))
    t0 = time.perf_counter()
    for _ in range(ps_steps):
        for hh, (l1, g1) in zip(hs, outs):
            spg.spingp_logml_grad(hh._h, l1, g1)
    torch.cuda.synchronize()
    el_s = (time.perf_counter() - t0) / ps_steps
    for hh in hs:
        hh.close()
    return {"workload": w.name, "n_series": S, "n_points": n, "points_per_s": n / el_b, "ms_per_step": 1e3 * el_b,
            "tile": {"R": R, "L": L}, "launch": "eager, side stream", "steps": steps,
            "graph_replay": {"ms_per_step": 1e3 * el_g, "points_per_s": n / el_g,
                             "launch": "one HIP graph of the forward + backward launches, replayed"},
            "per_series_launch": {"points_per_s": n / el_s, "ms_per_step": 1e3 * el_s, "steps": ps_steps},
            "speedup": el_s / el_b}


def forward_report(spg, steps, warmup):
    """The forward-only workload of Matern-5/2 at N = 2^20 (Exp(1) gaps, l = 5, var = 2,
    s2 = 0.05): per step the factorisation (cyclic reduction), logML with data fit and log det,
    posterior mean and selected-inverse variances (spingp_factor, spingp_logml, spingp_solve,
    spingp_selinv), eager launches on a side stream, tile from the autotuner of logML + gradient;
    with the per-kernel event times of one more pass."""
    import torch
    from paper_1610_08035_amd.spingp import spingp_profile, spingp_profile_read
    from workloads import make_config
    w = make_config(2)
    t, y, hyp = w.series(0)
    n = t.shape[0]
    dev = torch.device("cuda:0")
    td, yd, hd = (torch.as_tensor(a, device=dev) for a in (t, y, hyp))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    h = spg.Handle(w.terms, n, stream=side)
    h.assemble(td, yd, hd, autotune=True)
    ll, fit, ld = (torch.empty(1, dtype=torch.float64, device=dev) for _ in range(3))
    fm = torch.empty(n, dtype=torch.float64, device=dev)
    fv = torch.empty(n, dtype=torch.float64, device=dev)

    def step():
        spg.spingp_factor(h._h)
        spg.spingp_logml(h._h, ll, fit, ld)
        spg.spingp_solve(h._h, fm)
        spg.spingp_selinv(h._h, fv)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if h.status()[0] != 0:
        raise RuntimeError("forward workload failed validation")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    spingp_profile(h._h, 1)
    for _ in range(steps):
        step()
    prof = spingp_profile_read(h._h)
    spingp_profile(h._h, 0)
    torch.cuda.synchronize()
    R, L = spg.spingp_tile_shape(h.tile)
    h.close()
    return {"workload": "matern52_n1048576_exp1gaps_forward_factor_logml_mean_var", "n_points": n,
            "points_per_s": n / el, "ms_per_step": 1e3 * el, "steps": steps, "tile": {"R": R, "L": L},
            "launch": "eager, side stream",
            "kernel_ms_per_step": {k: round(v[0] / steps, 5) for k, v in prof.items() if v[1]},
            "logml": float(ll.item())}


def large_report(spg, steps, warmup):
    """The large single series (Matern-5/2, N = 2^24, Exp(1) gaps): logML + gradient throughput
    and the device memory the call holds (inputs, library workspace, outputs) next to what
    storing every reduction level would take (two elements of 33 doubles per node at b = 3)."""
    import torch
    from workloads import make_config
    w = make_config(5)
    n = w.n_points
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    td, yd = torch.as_tensor(w.t, device=dev), torch.as_tensor(w.y, device=dev)
    hd = torch.as_tensor(w.hyper.reshape(-1), device=dev)
    torch.cuda.synchronize()
    h = spg.Handle(w.terms, n, stream=torch.cuda.Stream())
    h.assemble(td, yd, hd, autotune=True)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, 3, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    if h.status()[0] != 0:
        raise RuntimeError("large workload failed validation")
    t0 = time.perf_counter()
    for _ in range(steps):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ws = h.workspace_bytes()
    R, L = spg.spingp_tile_shape(h.tile)
    h.close()
    return {"workload": "matern52_n16777216_exp1gaps_logml_grad", "n_points": n, "points_per_s": n / el,
            "tile": {"R": R, "L": L}, "launch": "eager, side stream",
            "ms_per_step": 1e3 * el, "steps": steps, "device_bytes_in_use": used, "workspace_bytes": ws,
            "input_bytes": 16 * n, "every_level_stored_bytes": 2 * 33 * 8 * n}


def _wide_report(spg, name, terms, t, y, hyper, steps, warmup):
    """logML + gradient of one series on the wide-state path (eager launches on a side stream),
    with the per-phase times from the library's events on one extra call."""
    import torch
    from paper_1610_08035_amd.spingp import spingp_profile, spingp_profile_read
    n = t.shape[0]
    dev = torch.device("cuda:0")
    td, yd = torch.as_tensor(t, device=dev), torch.as_tensor(y, device=dev)
    hd = torch.as_tensor(np.asarray(hyper, dtype=np.float64).reshape(-1), device=dev)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    h = spg.Handle(terms, n, stream=side)
    h.assemble(td, yd, hd)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, h.n_hyper, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    if h.status()[0] != 0:
        raise RuntimeError(f"{name} failed validation")
    # per-phase times from the library's events, then the timed steps without them
    spingp_profile(h._h, 1)
    spg.spingp_logml_grad(h._h, ll, g)
    prof = spingp_profile_read(h._h)
    spingp_profile(h._h, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        spg.spingp_logml_grad(h._h, ll, g)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    b, nh = h.b, h.n_hyper
    h.close()
    phases = {"leaves_up_sweep": prof["fwd_fold_tree"][0], "root": prof["top_tree"][0],
              "down_sweep_node_step": prof["bwd_elim_adjoint"][0], "gradient_sum": prof["series_reduce"][0]}
    return {"workload": name, "n_points": n, "state_dim": b, "n_hyper": nh,
            "points_per_s": n / el, "ms_per_step": 1e3 * el, "steps": steps, "launch": "eager, side stream",
            "phase_ms": {k: round(v, 4) for k, v in phases.items()}}


def sum_report(spg, steps, warmup):
    """Matern-3/2 + periodic with 3 harmonics (b = 10), N = 2^18, t uniform on [0, 1e4]:
    logML + the six-component gradient through the wide-state path (eager launches on a side
    stream; graph replay measures the same here)."""
    from workloads import make_config
    w = make_config(3)
    return _wide_report(spg, w.name + "_logml_grad", w.terms, w.t, w.y, w.hyper[0], steps, warmup)


def co2_report(spg, steps, warmup):
    """The three-term kernel of the CO2 fit: Matern-3/2 + quasi-periodic (3 harmonics) +
    squared exponential of order 6 (b = 16), N = 2^18 points uniform over 2^18 / 52 years,
    hyperparameters (0.8, 0.3, 1, 4, 1, 60, 8, 20, 0.05): logML + the nine-component gradient."""
    from workloads import KIND_MATERN32, KIND_QUASIPERIODIC, KIND_SQEXP
    from workloads.generate import make_series
    terms = [(KIND_MATERN32, 0), (KIND_QUASIPERIODIC, 3), (KIND_SQEXP, 6)]
    n = 1 << 18
    rng = np.random.default_rng(16)
    t = np.sort(rng.uniform(0.0, n / 52.0, n))
    hy = np.array([0.8, 0.3, 1.0, 4.0, 1.0, 60.0, 8.0, 20.0, 0.05])
    y = make_series(t, terms, hy, rng)
    return _wide_report(spg, "matern32+quasiperiodic3+sqexp6_n262144_weekly_logml_grad", terms, t, y, hy,
                        steps, warmup)


def predict_report(spg, steps, warmup):
    """Prediction at 2^16 new times (uniform over the data range) from the N = 2^20 Matern-5/2
    series: latent mean and variance through the merged chain (eager launches)."""
    import torch
    from workloads import make_config
    w = make_config(2)
    t, y, hyp = w.series(0)
    dev = torch.device("cuda:0")
    m = 1 << 16
    ts = torch.as_tensor(np.sort(np.random.default_rng(7).uniform(t[0], t[-1], m)), device=dev)
    td, yd, hd = (torch.as_tensor(a, device=dev) for a in (t, y, hyp))
    torch.cuda.synchronize()
    h = spg.Handle(w.terms, t.shape[0] + m, stream=torch.cuda.Stream())
    h.assemble(td, yd, hd)
    fm = torch.empty(m, dtype=torch.float64, device=dev)
    fv = torch.empty_like(fm)
    for _ in range(warmup):
        spg.spingp_predict(h._h, ts, fm, fv)
    torch.cuda.synchronize()
    if h.status()[0] != 0:
        raise RuntimeError("prediction workload failed validation")
    t0 = time.perf_counter()
    for _ in range(steps):
        spg.spingp_predict(h._h, ts, fm, fv)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    h.close()
    return {"workload": "matern52_n1048576_predict_65536", "n_train": int(t.shape[0]), "n_star": m,
            "ms_per_call": 1e3 * el, "merged_points_per_s": (t.shape[0] + m) / el, "steps": steps}


# Wide-path models of the block-size sweep: (b, terms, hyperparameter row) with kind codes
# 1 M32, 2 M52, 3 periodic, 4 M12, 5 M72, 6 quasi-periodic, 7 squared exponential; b = 10 is
# the sum kernel, b = 12 the paper's Matern-3/2 + 10th-order squared exponential, b = 16 the
# three-term CO2 kernel.
BSWEEP_WIDE = [
    (2, [(4, 0), (4, 0)], [3.0, 0.5, 20.0, 1.0, 0.05]),
    (3, [(4, 0), (1, 0)], [3.0, 0.5, 20.0, 1.0, 0.05]),
    (4, [(7, 4)], [8.0, 1.0, 0.05]),
    (5, [(1, 0), (2, 0)], [3.0, 0.5, 20.0, 1.0, 0.05]),
    (6, [(1, 0), (7, 4)], [3.0, 0.5, 8.0, 1.0, 0.05]),
    (7, [(2, 0), (3, 1)], [20.0, 1.0, 1.0, 0.8, 10.0, 0.05]),
    (8, [(1, 0), (7, 6)], [3.0, 0.5, 8.0, 1.0, 0.05]),
    (9, [(2, 0), (7, 6)], [3.0, 0.5, 8.0, 1.0, 0.05]),
    (10, [(1, 0), (3, 3)], [5.0, 2.0, 1.0, 1.0, 10.0, 0.05]),
    (11, [(1, 0), (2, 0), (6, 2)], [3.0, 0.5, 20.0, 1.0, 1.0, 0.7, 10.0, 60.0, 0.05]),
    (12, [(1, 0), (7, 10)], [3.0, 0.5, 8.0, 1.0, 0.05]),
    (13, [(2, 0), (7, 10)], [3.0, 0.5, 8.0, 1.0, 0.05]),
    (14, [(1, 0), (6, 1), (7, 8)], [3.0, 0.5, 1.0, 0.7, 10.0, 60.0, 8.0, 1.0, 0.05]),
    (15, [(4, 0), (6, 3), (7, 6)], [3.0, 0.5, 1.0, 0.7, 10.0, 60.0, 8.0, 1.0, 0.05]),
    (16, [(1, 0), (6, 3), (7, 6)], [0.8, 0.3, 1.0, 4.0, 1.0, 60.0, 8.0, 20.0, 0.05]),
]


def bsweep_report(spg, steps, warmup):
    """Block size sweep in the manner of the paper's time-versus-b experiment: logML + gradient
    per call for Matern nu = 1/2 .. 7/2 on the per-lane path (b = 1 .. 4, N = 1000 and 2^20) and
    for a sum of terms on the wide-state path at every b = 2 .. 16 (N = 1000 and 2^18; t with unit
    mean spacing, data drawn from the model), eager launches on a side stream."""
    import torch
    from workloads import KIND_MATERN12, KIND_MATERN32, KIND_MATERN52, KIND_MATERN72, make_batch
    from workloads.generate import make_series
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    rows = []
    cases = [(1, [(KIND_MATERN12, 0)], None, "lane"), (2, [(KIND_MATERN32, 0)], None, "lane"),
             (3, [(KIND_MATERN52, 0)], None, "lane"), (4, [(KIND_MATERN72, 0)], None, "lane")]
    cases += [(b, terms, hy, "wide") for b, terms, hy in BSWEEP_WIDE]
    for b, terms, hy, path in cases:
        for n in (1000, (1 << 20) if path == "lane" else (1 << 18)):
            if path == "lane":
                w = make_batch([n], np.array([[5.0, 2.0, 0.05]]), terms, seed=b)
                t, y, hyp = w.series(0)
            else:
                rng = np.random.default_rng(100 + b)
                t = np.sort(rng.uniform(0.0, float(n), n))
                hyp = np.asarray(hy, dtype=np.float64)
                y = make_series(t, terms, hyp, rng)
            td, yd, hd = (torch.as_tensor(a, device=dev) for a in (t, y, hyp))
            torch.cuda.synchronize()
            h = spg.Handle(terms, n, stream=side)
            h.assemble(td, yd, hd, autotune=path == "lane")
            ll = torch.empty(1, dtype=torch.float64, device=dev)
            g = torch.empty(1, h.n_hyper, dtype=torch.float64, device=dev)
            for _ in range(warmup):
                spg.spingp_logml_grad(h._h, ll, g)
            torch.cuda.synchronize()
            k = steps if n <= (1 << 16) or path == "lane" else max(2, steps // 10)
            t0 = time.perf_counter()
            for _ in range(k):
                spg.spingp_logml_grad(h._h, ll, g)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / k
            rows.append({"b": b, "path": path, "terms": [list(x) for x in terms], "n_points": n,
                         "ms_per_call": 1e3 * el, "points_per_s": n / el,
                         "tile": dict(zip(("R", "L"), spg.spingp_tile_shape(h.tile))) if path == "lane" else "wide"})
            h.close()
    return rows


def fit_report(spg):
    """Maximum-marginal-likelihood fits by scaled conjugate gradients: the N = 2^20 Matern-5/2
    series from a start away from the generating hyperparameters (l = 5, var = 2, s2 = 0.05),
    and CO2-shaped stand-ins (weekly grid; Matern-3/2 + quasi-periodic, and the full three-term
    model with the squared-exponential trend): evaluations, wall time, time per evaluation (one
    logML + gradient call plus the host round trip)."""
    import torch
    from paper_1610_08035_amd.optimize import fit
    from workloads import make_config
    w = make_config(2)
    t, y, hyp = w.series(0)
    dev = torch.device("cuda:0")
    td, yd = torch.as_tensor(t, device=dev), torch.as_tensor(y, device=dev)
    h = spg.Handle(w.terms, t.shape[0], stream=torch.cuda.Stream())
    hyper0 = [2.0, 1.0, 0.2]
    fit(td, yd, w.terms, hyper0, max_iter=3, handle=h)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fit(td, yd, w.terms, hyper0, handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.close()
    out = [{"workload": "matern52_n1048576_fit_scg", "start": hyper0, "hyper": [float(v) for v in res.hyper[0]],
            "logml": float(res.logml[0]), "converged": res.converged, "iterations": res.n_iter,
            "evaluations": res.n_eval, "seconds": el, "ms_per_evaluation": 1e3 * el / res.n_eval}]
    # a stand-in shaped like the paper's CO2 fit: 2195 weekly points (years), Matern-3/2 +
    # quasi-periodic, seven hyperparameters, data drawn from (8, 4, 1, 2, 1, 30, 0.1)
    from workloads import KIND_MATERN32, KIND_QUASIPERIODIC
    from workloads.generate import make_series
    terms = [(KIND_MATERN32, 0), (KIND_QUASIPERIODIC, 3)]
    t = np.arange(2195) / 52.0
    y = make_series(t, terms, np.array([8.0, 4.0, 1.0, 2.0, 1.0, 30.0, 0.1]), np.random.default_rng(2195))
    td, yd = torch.as_tensor(t, device=dev), torch.as_tensor(y, device=dev)
    hyper0 = [5.0, 2.0, 0.8, 1.0, 1.01, 50.0, 0.2]
    h = spg.Handle(terms, t.shape[0], stream=torch.cuda.Stream())
    fit(td, yd, terms, hyper0, max_iter=3, handle=h)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fit(td, yd, terms, hyper0, max_iter=2000, handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.close()
    out.append({"workload": "co2_shaped_weekly2195_matern32+quasiperiodic3_fit_scg", "start": hyper0,
                "hyper": [float(v) for v in res.hyper[0]], "logml": float(res.logml[0]),
                "converged": res.converged, "iterations": res.n_iter, "evaluations": res.n_eval,
                "seconds": el, "ms_per_evaluation": 1e3 * el / res.n_eval})
    # the full three-term model (Matern-3/2 + quasi-periodic + squared-exponential trend, b = 16,
    # nine hyperparameters), data drawn from (0.8, 0.3, 1, 4, 1, 60, 8, 20, 0.05)
    from workloads import KIND_SQEXP
    terms = [(KIND_MATERN32, 0), (KIND_QUASIPERIODIC, 3), (KIND_SQEXP, 6)]
    y = make_series(t, terms, np.array([0.8, 0.3, 1.0, 4.0, 1.0, 60.0, 8.0, 20.0, 0.05]), np.random.default_rng(2196))
    yd = torch.as_tensor(y, device=dev)
    hyper0 = [1.0, 0.5, 0.9, 2.0, 1.005, 40.0, 10.0, 10.0, 0.1]
    h = spg.Handle(terms, t.shape[0], stream=torch.cuda.Stream())
    fit(td, yd, terms, hyper0, max_iter=3, handle=h)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fit(td, yd, terms, hyper0, max_iter=3000, handle=h)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.close()
    out.append({"workload": "co2_shaped_weekly2195_matern32+quasiperiodic3+sqexp6_fit_scg", "start": hyper0,
                "hyper": [float(v) for v in res.hyper[0]], "logml": float(res.logml[0]),
                "converged": res.converged, "iterations": res.n_iter, "evaluations": res.n_eval,
                "seconds": el, "ms_per_evaluation": 1e3 * el / res.n_eval})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-series batched report")
    ap.add_argument("--no-large", action="store_true", help="skip the N = 2^24 report")
    ap.add_argument("--no-sum", action="store_true", help="skip the b = 10 sum-kernel report")
    ap.add_argument("--no-co2", action="store_true", help="skip the b = 16 three-term (CO2 kernel) report")
    ap.add_argument("--no-predict", action="store_true", help="skip the prediction report")
    ap.add_argument("--no-fit", action="store_true", help="skip the hyperparameter-fit report")
    ap.add_argument("--no-bsweep", action="store_true", help="skip the block-size sweep")
    ap.add_argument("--no-forward", action="store_true", help="skip the forward-only (factor, logML, mean, "
                    "variance) report")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the CPU oracle on every workload (minutes) and print its JSON")
    ap.add_argument("--tile", type=int, default=None,
                    help="headline tile shape index instead of the autotuner's choice (counter runs)")
    ap.add_argument("--only", choices=["batched", "large", "sum", "co2", "predict", "fit", "bsweep", "forward"],
                    default=None,
                    help="run one secondary workload alone and print its JSON (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scales the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X; "
              "multi-GPU runs are not part of this benchmark", file=sys.stderr)
        sys.exit(2)

    if args.cpu_table:
        print(json.dumps({"cpu_table": cpu_table()}), flush=True)
        return
    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 5}))
        return
    import paper_1610_08035_amd as spg
    from paper_1610_08035_amd.spingp import spingp_profile, spingp_profile_read
    from workloads import make_config
    if args.only:
        if args.only == "fit":
            print(json.dumps({"fit": fit_report(spg)}), flush=True)
            return
        fn = {"batched": batched_report, "large": large_report, "sum": sum_report, "co2": co2_report,
              "predict": predict_report, "bsweep": bsweep_report, "forward": forward_report}[args.only]
        print(json.dumps({args.only: fn(spg, args.steps, args.warmup)}), flush=True)
        return

    w = make_config(2)              # Matern-5/2, N = 2^20, Exp(1) gaps, l = 5, var = 2, s2 = 0.05
    n = w.n_points
    t, y, hyp = w.series(0)
    dev = torch.device("cuda:0")
    td = torch.as_tensor(t, device=dev)
    yd = torch.as_tensor(y, device=dev)
    hd = torch.as_tensor(hyp, device=dev)
    torch.cuda.synchronize()
    # All launches go to a side stream of default priority: back-to-back eager launches there
    # keep the GPU busy (the host enqueues a step in about 12 us, the GPU runs it in about
    # 100 us), while a graph replay or the legacy default stream adds a gap of several us per
    # step.  The graph replay is timed as well and reported beside the main number.
    side = torch.cuda.Stream()
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, 3, dtype=torch.float64, device=dev)
    hs = spg.Handle(w.terms, n, stream=side)
    if args.tile is None:
        hs.assemble(td, yd, hd, autotune=True)   # tile shape timed by the library's autotuner
    else:
        hs.tile = args.tile
        hs.assemble(td, yd, hd)

    def step():
        spg.spingp_logml_grad(hs._h, ll, g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rc, bad = hs.status()
    if rc != 0:
        raise RuntimeError(f"device status {rc} at {bad}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same steps as HIP-graph replays (same stream, same tile)
    hg = spg.Handle(w.terms, n, stream=side)
    hg.tile = hs.tile
    hg.assemble(td, yd, hd, graph=True)
    for _ in range(args.warmup):
        spg.spingp_logml_grad(hg._h, ll, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        spg.spingp_logml_grad(hg._h, ll, g)
    torch.cuda.synchronize()
    el_graph = (time.perf_counter() - t0) / args.steps
    hg.close()
    # per-kernel averages: the same steps with HIP events around each kernel on the side stream
    h = spg.Handle(w.terms, n, stream=side)
    h.tile = hs.tile
    h.assemble(td, yd, hd)
    for _ in range(2):
        spg.spingp_logml_grad(h._h, ll, g)
    spingp_profile(h._h, 1)
    for _ in range(args.steps):
        spg.spingp_logml_grad(h._h, ll, g)
    prof = spingp_profile_read(h._h)
    spingp_profile(h._h, 0)
    spg.spingp_logml_grad(hs._h, ll, g)
    torch.cuda.synchronize()
    hs.close()

    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    per_kernel = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    dom = max(FLOPS_PER_POINT, key=lambda k: per_kernel[k])
    t_dom = per_kernel[dom] * 1e-3
    achieved = FLOPS_PER_POINT[dom] * n / t_dom / 1e12
    traffic = None
    if TRAFFIC["kernel"] == dom and TRAFFIC["source_sha"] == kernel_source_sha():
        traffic = TRAFFIC["bytes"].get(tuple(spg.spingp_tile_shape(h.tile)))
    # the binding roof from the algorithmic intensity (flop per byte of t, y) against the machine
    # balance; beside it the HBM rate of the measured traffic (counters), when it is current
    intensity = FLOPS_PER_POINT[dom] / ALG_BYTES_PER_POINT[dom]
    bound = "alu" if intensity > MACHINE_BALANCE else "hbm"
    hbm = {"algorithmic_bytes_per_launch": ALG_BYTES_PER_POINT[dom] * n,
           "algorithmic_GBs": ALG_BYTES_PER_POINT[dom] * n / t_dom / 1e9, "peak_GBs": PEAK_HBM_GBS}
    hbm["algorithmic_frac"] = hbm["algorithmic_GBs"] / PEAK_HBM_GBS
    if traffic is not None:
        hbm["measured_bytes_per_launch"] = traffic
        hbm["measured_GBs"] = traffic / t_dom / 1e9
        hbm["measured_frac"] = hbm["measured_GBs"] / PEAK_HBM_GBS
        hbm["measured_intensity_flop_per_byte"] = FLOPS_PER_POINT[dom] * n / traffic
        hbm["source"] = "rocprofv3 FETCH_SIZE and WRITE_SIZE per launch, scaled by a device copy of known size"
    out = {
        "metric": "time points/sec, logML+grad, Matern-5/2 N=2^20 FP64; % HBM roofline",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded GP prior sample + noise, Exp(1) gaps)",
        "config": {"workload": "matern52_n1048576_exp1gaps_logml_grad", "n_points": n, "state_dim": 3,
                   "n_hyper": 3, "hyper": [float(v) for v in hyp], "launch": "eager, side stream",
                   "tile": dict(zip(("R", "L"), spg.spingp_tile_shape(h.tile))),
                   "cache": "inputs and workspace (about 80 MB) stay resident in the 256 MB MALL between steps"},
        "graph_replay": {"ms_per_step": 1e3 * el_graph, "points_per_s": n / el_graph},
        "roofline": {"bound": bound, "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_point": FLOPS_PER_POINT[dom],
                     "algorithmic_intensity_flop_per_byte": intensity, "machine_balance_flop_per_byte": MACHINE_BALANCE,
                     "hbm": hbm},
        "kernel_ms": {k: round(v, 5) for k, v in per_kernel.items()},
        "logml": float(ll.item()),
    }
    h.close()
    if not args.no_forward:
        out["forward"] = forward_report(spg, args.steps, args.warmup)
    if not args.no_batched:
        out["batched"] = batched_report(spg, args.steps, args.warmup)
    if not args.no_large:
        out["large"] = large_report(spg, max(2, args.steps // 4), max(1, args.warmup // 2))
    if not args.no_sum:
        out["sum_kernel"] = sum_report(spg, max(2, args.steps // 4), max(1, args.warmup // 2))
    if not args.no_co2:
        out["co2_kernel"] = co2_report(spg, max(2, args.steps // 10), 1)
    if not args.no_predict:
        out["predict"] = predict_report(spg, max(2, args.steps // 4), max(1, args.warmup // 2))
    if not args.no_fit:
        out["fit"] = fit_report(spg)
    if not args.no_bsweep:
        out["bsweep"] = bsweep_report(spg, max(2, args.steps // 4), max(1, args.warmup // 2))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        out["cpu_config1"] = cpu_config1()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
