"""Benchmark of the fused D2Q9 interface-capturing step on one MI355X.

Workload (default): single vortex on an 8192 x 8192 periodic lattice, disk
R = 0.15 N at (0.5 N, 0.75 N), eps = 1, tau = 0.8, delta = 1e-10, U = 0.02,
period T = 4096 steps; FP32 collide with FP32 population storage.  W warm-up
steps run first on a separate context; the timed run then starts from the
initial field and covers K steps, so with K = T the L2 shape error is taken
at the return time t = T.

Prints ONE JSON line: MLUPS (whole job), the step kernel's achieved HBM
bandwidth against the 8 TB/s peak (algorithmic bytes: every stored value
read and written once per launch; the two-step kernel takes two steps per
launch), the L2 shape error, the same run with the 16-bit shifted storage
forms, and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed instructions (which this build does not
# use): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s,
# 78.6 TFLOP/s with an FMA counted as two operations (the 157.3 TFLOP/s
# figure counts packed FMAs, two per lane); the VALU issues 1024 SIMDs x 2.4
# GHz / 4 cycles = 614.4 G wave64 instructions/s
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
# algorithmic HBM bytes per node-update of the FP32 form: nine populations
# read and written once (Sec. 2.2, Eq. (9))
BYTES_PER_NODE_UPDATE = 72.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "step_f32_8192_hbm_counters.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "step_f32_8192_sq_counters.txt")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbac_kernels.hpp", "lbac.hip"):
        with open(os.path.join(ROOT, "paper_2203_05230_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _summary_fields(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def _counter_summary(path, key, launch):
    """A value from a committed rocprofv3 counter summary, if the summary was
    taken on the current kernel source in the same launch shape (tile width,
    strip height and variant: the strip height changes the rows re-read
    between strips, hence the fetched bytes); else None."""
    try:
        kv = _summary_fields(path)
        if kv.get("kernel_source_sha") != kernel_source_hash():
            return None
        shape = tuple(int(v) for v in kv["launch"].split(","))
        if launch is None or shape != tuple(int(v) for v in launch):
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def profiled_launch():
    """The launch shape (bx, strip_h, variant) the committed counter summary
    of the step kernel was taken on (the shape the autotuner picked on the
    profiling run), if it was taken on the current kernel source; else None."""
    try:
        kv = _summary_fields(COUNTERS_FILE)
        if kv.get("kernel_source_sha") != kernel_source_hash():
            return None
        return tuple(int(v) for v in kv["launch"].split(","))
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(launch):
    """HBM bytes per step-kernel launch (FETCH_SIZE and WRITE_SIZE, scaled by a
    plain copy's readings), or None."""
    return _counter_summary(COUNTERS_FILE, "hbm_bytes_per_launch", launch)


def measured_valu_instructions(launch):
    """SQ_INSTS_VALU (wave instructions) per step-kernel launch, or None."""
    return _counter_summary(SQ_FILE, "valu_instructions_per_launch", launch)


def measured_fp32_flops(launch):
    """FP32 operations per step-kernel launch counted by the SQ counters:
    64 lanes x (ADD + MUL + TRANS + 2 FMA wave instructions), or None."""
    return _counter_summary(SQ_FILE, "fp32_flops_per_launch", launch)


def run_form(lbac, torch, case, phi0, precision, steps, warmup, launch=None, autotune=False, graph=0, keep_phi=False):
    # a stream of our own: the library works on it and the events are recorded
    # on it (torch's default stream has handle 0, which the library would
    # replace by a private stream)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    assert stream.cuda_stream != 0
    c = {**case, "precision": precision}
    sim = lbac.Simulation(c, phi0, stream=stream.cuda_stream)
    if launch:
        sim.set_launch(*launch)
    if autotune:
        sim.autotune(12)
    launch = sim.get_launch()
    if warmup:
        sim.step(warmup)
    torch.cuda.synchronize()
    sim.close()
    # timed run from the initial field
    sim = lbac.Simulation(c, phi0, stream=stream.cuda_stream)
    sim.set_launch(*launch)
    if graph:
        sim.set_graph_chunk(graph)
    m0 = sim.mass()
    spl = sim.steps_per_launch()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    evm = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    # the S-step launches, then the one-step launches of the remainder: the
    # first interval times the dominant kernel alone
    ev0.record(stream)
    sim.step(steps - steps % spl)
    evm.record(stream)
    sim.step(steps % spl)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    full_launches = steps // spl
    launch_ms = ev0.elapsed_time(evm) / full_launches if full_launches else None
    e1, e2 = sim.shape_error(phi0)
    m1 = sim.mass()
    assert sim.stream() == stream.cuda_stream
    # practical ceiling: the same bytes moved in the step's access pattern by a plain copy
    copy_us = sim.copy_ceiling(20)
    out = dict(ms_total=ms, wall_s=wall, launch=list(launch), e1=e1, e2=e2, mass_drift=abs(m1 - m0) / m0,
               bytes_per_node=sim.bytes_per_node(), steps_per_launch=spl, t_end=sim.time(),
               copy_us=copy_us, launch_ms=launch_ms, full_launches=full_launches, mass=m1)
    if keep_phi:
        out["phi"] = sim.phi()
    sim.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    return out


def batch_leg(lbac, torch, W, count, seed, strip_h=None, seq_cap=512, precision="f32"):
    """The batched form on the seeded instance list (sides 128..512, eps in
    {0.5, 1, 2}, tau in [0.6, 1]; half single vortex over one period of 8 N
    steps, half slotted disk over one revolution of 64 N steps), every
    instance advanced over its whole run in one run of the batch (instances
    retire at their own step counts).  Reports the aggregate rate, each
    instance's E2 against its phi0 at t = T, four instances checked bitwise
    against the same instance advanced alone, and, for context, the rate of
    the list advanced one instance after another through lbac_step (three
    steps per launch, HIP-graph replay) over the first `seq_cap` steps of
    each instance.  strip_h: rows per item, else autotuned (dry runs).
    precision: the batch's storage; with 16-bit storage the sequential
    context rate is skipped (seq_cap 0)."""
    cases = W.batch_cases(count=count, seed=seed)
    phis = [W.initial_field(c) for c in cases]
    steps = [c["steps"] for c in cases]
    updates = float(sum(c["nx"] * c["ny"] * k for c, k in zip(cases, steps)))
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    b = lbac.Batch(cases, phis, stream=stream.cuda_stream, precision=precision)
    if strip_h:
        b.set_shape(strip_h)
    else:
        # dry runs (the instances' state is kept) of the real step counts scaled
        # by 1/16: the same retirement order, so the tail is tuned for too
        b.autotune([max(3, k // 16) for k in steps])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.run(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1)
    e2 = []
    for k in range(count):
        inst = b.instance(k)
        assert inst.time() == steps[k]
        e2.append(inst.shape_error(phis[k])[1])
    kinds = ["vortex" if c["vel"] == "vortex" else "slotted disk" for c in cases]
    probe = sorted({0, count // 2 - 1, count // 2, count - 1})
    got = {k: b.instance(k).phi() for k in probe}
    shape = b.get_shape()
    b.close()

    def alone(k, n):
        sim = lbac.Simulation({**cases[k], "precision": precision}, phis[k], stream=stream.cuda_stream)
        sim.set_launch(224, 40, 4)
        sim.set_graph_chunk(96)
        sim.step(n)
        return sim

    same = True
    for k in probe:
        sim = alone(k, steps[k])
        same = same and bool(np.array_equal(got[k], sim.phi()))
        sim.close()
    mlups = updates / (ms_batch * 1e-3) / 1e6
    seq = None
    if seq_cap > 0:
        # sequential context rate: the first seq_cap steps of every instance, one after another
        sims = [alone(k, 0) for k in range(count)]
        for sim in sims:
            sim.step(96)  # captures the graph outside the timed region
        torch.cuda.synchronize()
        seq_steps = [max(0, min(k, seq_cap) - 96) for k in steps]
        seq_updates = float(sum(c["nx"] * c["ny"] * k for c, k in zip(cases, seq_steps)))
        ev0.record(stream)
        for sim, k in zip(sims, seq_steps):
            sim.step(k)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_seq = ev0.elapsed_time(ev1)
        for sim in sims:
            sim.close()
        seq = dict(mlups=round(seq_updates / (ms_seq * 1e-3) / 1e6, 1), ms=round(ms_seq, 2),
                   steps_per_instance_cap=seq_cap, launch=[224, 40, 4], graph_chunk=96)
    torch.cuda.set_stream(torch.cuda.default_stream())
    e2a = np.array(e2)
    by_kind = {kind: dict(instances=int(sum(1 for x in kinds if x == kind)),
                          e2_median=float(np.median(e2a[[x == kind for x in kinds]])),
                          e2_max=float(np.max(e2a[[x == kind for x in kinds]])))
               for kind in ("vortex", "slotted disk")}
    out = dict(instances=count, seed=seed, precision=precision, node_updates=updates, steps_min=min(steps),
               steps_max=max(steps), mlups=round(mlups, 1), ms=round(ms_batch, 2), strip_h=shape[0],
               resident_workgroups=shape[1], e2_at_T=by_kind, e2_per_instance=[float("%.4e" % v) for v in e2],
               bitwise_equal_probe=same, probed=probe)
    if seq is not None:
        out.update(sequential=seq, speedup_vs_sequential=round(mlups / seq["mlups"], 3))
    return out


CLOSURE_LAUNCHES = ((224, 40, 4), (192, 40, 4), (160, 40, 4), (224, 80, 4), (224, 40, 3))


def closure_leg(lbac, torch, case, phi0, steps, theta=0.02, launch=None):
    """The step with the learned closure on the benchmark grid (BF16 MFMA
    inference on interface-band nodes inside the multi-step kernel's steps),
    with a seeded network; the cost depends on the band's size, not on the
    weights' values.  The launch shape is the fastest of a few multi-step
    shapes on 24 steps (or `launch`); also reported: the one-step path (step
    kernel, band list and correction pass) for context."""
    from paper_2203_05230_amd import closure as CL

    w = CL.init_weights(7, out_scale=1e-3)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(shape, k):
        sim = lbac.Simulation({**case, "precision": "f32"}, phi0, stream=stream.cuda_stream)
        sim.set_launch(*shape)
        sim.set_closure(w, theta=theta)
        sim.step(6)
        torch.cuda.synchronize()
        ev0.record(stream)
        sim.step(k)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / k
        return sim, ms

    tried = {}
    if launch is None:
        for shape in CLOSURE_LAUNCHES:
            sim, ms = timed(shape, 24)
            sim.close()
            tried[",".join(map(str, shape))] = round(ms, 4)
        launch = min(CLOSURE_LAUNCHES, key=lambda sh: tried[",".join(map(str, sh))])
    sim, ms = timed(launch, steps)
    phi = sim.phi()
    spl = sim.steps_per_launch()
    sim.close()
    pc = np.clip(phi, 0.0, 1.0)
    band = int(((pc > theta) & (pc < 1.0 - theta)).sum())
    sim1, ms1 = timed((256, 40, 2), 24)
    sim1.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    n = case["nx"] * case["ny"]
    return dict(steps=steps, launch=list(launch), steps_per_launch=spl, ms_per_step=round(ms, 4),
                mlups=round(n / (ms * 1e-3) / 1e6, 1), band_nodes=band, band_fraction=band / n,
                mac_per_band_node=5824, theta=theta, shapes_tried_ms_per_step=tried,
                one_step_path=dict(launch=[256, 40, 2], ms_per_step=round(ms1, 4),
                                   mlups=round(n / (ms1 * 1e-3) / 1e6, 1)))


def train_leg(lbac, torch, steps, batch=4096):
    """One Adam step of the closure network's training (forward, backward,
    gradient and update kernels) on a seeded synthetic batch of `batch`
    stencils (inputs uniform in [0, 1], targets normal with deviation 0.05),
    the batch size of the closure's training: time per step from HIP events
    over `steps` steps after 5 untimed ones."""
    from paper_2203_05230_amd import closure as CL

    rng = np.random.default_rng(1)
    X = torch.from_numpy(rng.uniform(0.0, 1.0, (batch, 25)).astype(np.float32)).cuda()
    Y = torch.from_numpy(rng.normal(0.0, 0.05, (batch, 2)).astype(np.float32)).cuda()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    net = lbac.Mlp(CL.init_weights(3), stream=stream.cuda_stream)
    for _ in range(5):
        net.train_step(X.data_ptr(), Y.data_ptr(), batch, 1e-3)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        net.train_step(X.data_ptr(), Y.data_ptr(), batch, 1e-3)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) / steps * 1e3
    loss = net.train_step(X.data_ptr(), Y.data_ptr(), batch, 1e-3, want_loss=True)
    torch.cuda.set_stream(torch.cuda.default_stream())
    # FP32 matrix work of one step: forward 2 (25 * 64 + 64 * 64 + 64 * 2)
    # per sample, backward about twice that
    flop = 3 * 2 * (25 * 64 + 64 * 64 + 64 * 2) * batch
    return dict(batch=batch, steps=steps, us_per_step=round(us, 2), samples_per_s=round(batch / (us * 1e-6), 1),
                fp32_tflops=round(flop / (us * 1e-6) / 1e12, 3), loss=loss)


def c2_leg(lbac, torch, W, n, steps):
    """The 1024^2 single vortex (R = 0.15 n at (0.5 n, 0.75 n), tau 0.8, U
    0.02, period = `steps`) at eps 0.5 and 1 with FP32, FP16 and BF16 shifted
    storage, each over one full period from phi0: MLUPS, E1 and E2 against
    phi0 at t = T, mass drift, E2 of each 16-bit form relative to FP32, and,
    where the FP64 oracle's phi(T) of the same run is stored
    (tests/golden/c2_oracle_*.npz, written by tests/golden/make_c2_oracle.py),
    the relative L2 distance to it and the mass difference from the oracle's.
    The state (75 MB for FP32) stays in the 256 MB last-level cache, so these
    rates are not HBM rates; the steps are replayed from captured HIP graphs
    of 96 steps."""
    out = {}
    for eps in (0.5, 1.0):
        case = W.single_vortex_case(n, eps=eps, tau=0.8, U=0.02, period_T=float(steps))
        phi0 = W.circle(n, eps)
        golden = os.path.join(ROOT, "tests", "golden", "c2_oracle_%d_eps%g.npz" % (n, eps))
        ref = None
        if os.path.exists(golden):
            z = np.load(golden)
            if int(z["steps"]) == steps:
                ref = (z["phi"].astype(np.float64), float(z["massT"]))
        runs = {}
        for prec in ("f32", "f32_f16store", "f32_bf16store"):
            r = run_form(lbac, torch, case, phi0, prec, steps, 64, autotune=True, graph=96, keep_phi=ref is not None)
            runs[prec] = dict(mlups=round(n * n * steps / (r["ms_total"] * 1e-3) / 1e6, 1), e2=r["e2"], e1=r["e1"],
                              mass_drift=r["mass_drift"], launch=r["launch"])
            if ref is not None:
                runs[prec]["rel_l2_vs_oracle"] = float(np.linalg.norm(r["phi"] - ref[0]) / np.linalg.norm(ref[0]))
                runs[prec]["mass_vs_oracle"] = abs(r["mass"] - ref[1]) / ref[1]
        for prec in ("f32_f16store", "f32_bf16store"):
            runs[prec]["e2_vs_f32"] = runs[prec]["e2"] / runs["f32"]["e2"]
        out["eps=%g" % eps] = runs
    return dict(grid=n, steps=steps, **out)


def c1_leg(lbac, torch, W, steps):
    """The 64^2 single vortex in FP64 (R = 9.6 at (32, 48), eps 1, tau 0.8, U
    0.02, period = `steps`), the parity configuration, over one period from
    phi0: E1, E2 and mass drift at t = T, and MLUPS with the launch shape
    autotuned and the steps replayed from captured HIP graphs of 100 steps
    (4096 nodes per step: latency- and launch-bound)."""
    case = W.single_vortex_case(64, eps=1.0, tau=0.8, U=0.02, period_T=float(steps))
    phi0 = W.circle(64, 1.0)
    r = run_form(lbac, torch, case, phi0, "f64", steps, 0, autotune=True, graph=100)
    return dict(grid=64, steps=steps, precision="f64", mlups=round(64 * 64 * steps / (r["ms_total"] * 1e-3) / 1e6, 1),
                e2=r["e2"], e1=r["e1"], mass_drift=r["mass_drift"], launch=r["launch"])


def leg_3d(lbac, torch, W, n, steps, launch=None):
    """The D3Q19 form on an n^3 ball in the deformation field (FP32 storage),
    launch shape autotuned (or given); timed on the library's stream."""
    case = dict(nx=n, ny=n, nz=n, eps=1.0, tau=0.8, delta=1e-10, vel="deformation", U=0.02,
                period_T=3.0 * n / 0.02, precision="f32")
    phi0 = W.sphere(n, 1.0, R_frac=0.15)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    sim = lbac.Simulation3(case, phi0, stream=stream.cuda_stream)
    if launch:
        sim.set_launch(*launch)
    else:
        sim.autotune(4)
    sim.step(4)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    m = sim.mass()
    bpn = sim.bytes_per_node()
    launch = sim.get_launch()
    sim.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    nodes = n ** 3
    return dict(grid=n, steps=steps, ms_per_step=round(ms, 4), mlups=round(nodes / (ms * 1e-3) / 1e6, 1),
                bytes_per_node=bpn, hbm_gbs_algorithmic=round(bpn * nodes / (ms * 1e-3) / 1e9, 1),
                mass_drift=abs(m - phi0.sum()) / phi0.sum(), launch=list(launch))


def _native_oracle():
    """The FP64 oracle compiled for the host that runs the benchmark (gcc -O3
    -march=native, as the CPU baseline asks; the in-tree build is portable
    -O2), loaded in place of the in-tree build; None if gcc is missing (the
    in-tree build is then timed and the record says so)."""
    import tempfile

    from oracle import build as OB
    from oracle import lib as O

    out = os.path.join(tempfile.gettempdir(), "liboracle_native_%d.so" % os.getpid())
    try:
        OB.build_native(out)
    except (OSError, RuntimeError) as e:
        print("bench: native oracle build failed (%s); timing the in-tree build" % e, file=sys.stderr, flush=True)
        return None
    O.use_library(out)
    return "gcc " + " ".join(OB.NATIVE_FLAGS)


def _oracle_rate(case, phi0, steps):
    """Seconds of stepping (set-up subtracted) of the FP64 oracle for `steps`
    steps of `case`, with whatever OpenMP thread count this process has."""
    from oracle import lib as O

    p = O.Params(case["nx"], case["ny"], eps=case["eps"], tau=case["tau"], delta=case["delta"],
                 vel_kind=O.VEL_VORTEX, U=case["U"], period_T=case["period_T"])
    O.lib()
    t0 = time.perf_counter()
    O.run(p, phi0, 0)  # set-up alone (allocation, initial populations)
    t1 = time.perf_counter()
    O.run(p, phi0, steps)
    t2 = time.perf_counter()
    return (t2 - t1) - (t1 - t0)


def _single_core_child(spec):
    """Child-process body of the single-core oracle leg: `spec` is "n,steps";
    prints one JSON object.  Runs with OMP_NUM_THREADS=1 and touches no GPU."""
    from paper_2203_05230_amd import workloads as W

    _native_oracle()
    n, steps = (int(v) for v in spec.split(","))
    case = W.single_vortex_case(n, eps=1.0, tau=0.8, U=0.02, period_T=4096.0)
    dt = _oracle_rate(case, W.circle(n, 1.0), steps)
    print(json.dumps({"n": n, "steps": steps, "seconds": dt}), flush=True)


def cpu_baseline(phi0, case, steps, single_core_n=2048, single_core_steps=4):
    """The FP64 oracle as it stands, on the host cores, for `steps` steps of the
    same grid (a bounded sample of the workload); plus the same oracle on one
    core, in a child process, over `single_core_steps` steps of the same
    vortex on a `single_core_n` grid (per-node rate; the grid still far exceeds
    the caches)."""
    flags = _native_oracle()
    dt = _oracle_rate(case, phi0, steps)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=case["nx"] * case["ny"] * steps / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
               sample="%d steps of the %dx%d single vortex (FP64 oracle, OpenMP over rows); %.1f s of "
               "stepping, set-up time subtracted" % (steps, case["nx"], case["ny"], dt),
               build=flags or "in-tree build (gcc -O2)")
    if single_core_steps > 0:
        import subprocess

        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-single-core",
                            "%d,%d" % (single_core_n, single_core_steps)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            sc = json.loads(r.stdout.strip().splitlines()[-1])
            out["single_core"] = dict(
                value=sc["n"] ** 2 * sc["steps"] / sc["seconds"] / 1e6, unit="MLUPS", cores=1,
                sample="%d steps of the %dx%d single vortex, one OpenMP thread; %.1f s of stepping"
                % (sc["steps"], sc["n"], sc["n"], sc["seconds"]))
        else:
            out["single_core"] = dict(error=r.stderr.strip().splitlines()[-1:] or ["exit %d" % r.returncode])
    # the oracle on the two smaller single-vortex configurations, for context:
    # 64^2 over its full 2000-step period and 1024^2 over 128 steps
    from paper_2203_05230_amd import workloads as W

    others = {}
    for n, period, nsteps in ((64, 2000.0, 2000), (1024, 16384.0, 128)):
        c = W.single_vortex_case(n, eps=1.0, tau=0.8, U=0.02, period_T=period)
        t = _oracle_rate(c, W.circle(n, 1.0), nsteps)
        others["%dx%d" % (n, n)] = dict(value=n * n * nsteps / t / 1e6, unit="MLUPS", steps=nsteps,
                                        seconds=round(t, 2))
    out["other_configs"] = others
    try:
        with open("/proc/cpuinfo") as fh:
            names = [ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")]
        out["cpu_model"] = names[0] if names else None
    except OSError:
        out["cpu_model"] = None
    out["host_cpus"] = os.cpu_count()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096)
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--eps", type=float, default=1.0)
    ap.add_argument("--period", type=float, default=4096.0)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--forms", default="f32_f16store,f32_bf16store",
                    help="extra storage forms timed on the same workload ('' for none)")
    ap.add_argument("--cpu-steps", type=int, default=16, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--cpu-single-core", default="", help=argparse.SUPPRESS)
    ap.add_argument("--batch", type=int, default=256, help="instances in the batched leg (0: skip)")
    ap.add_argument("--batch-strip", type=int, default=0, help="strip height of the batched leg (default: autotune)")
    ap.add_argument("--batch-f16", type=int, default=1, help="also time the batched list with FP16 storage (0: skip)")
    ap.add_argument("--closure-steps", type=int, default=256, help="steps of the closure leg (0: skip)")
    ap.add_argument("--train-steps", type=int, default=200, help="Adam steps of the closure-training leg (0: skip)")
    ap.add_argument("--grid3d", type=int, default=256, help="side of the D3Q19 leg (0: skip)")
    ap.add_argument("--c1-steps", type=int, default=2000, help="steps (= period) of the 64^2 FP64 run (0: skip)")
    ap.add_argument("--c2-steps", type=int, default=16384,
                    help="steps (= period) of the 1024^2 storage-form comparison (0: skip)")
    ap.add_argument("--launch", default="",
                    help="bx,strip_h,variant, or 'auto' to autotune (default: the shape the committed counters were "
                         "taken on, when they match the kernel source and the default workload; else autotune)")
    ap.add_argument("--one-step-steps", type=int, default=512,
                    help="steps of the one-step kernel timed for comparison when the two-step kernel runs (0: skip)")
    ap.add_argument("--steps3d", type=int, default=200, help="timed steps of the D3Q19 leg")
    ap.add_argument("--launch3d", default="", help="tile_x,tile_y,variant,strip_z,z_major of the D3Q19 leg (default: autotune)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (reference kernel for "
                         "scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.cpu_single_core:
        _single_core_child(args.cpu_single_core)
        return
    if args.copy_calibration:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (see the sharding notes "
              "in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2203_05230_amd import lbac, workloads as W

    lbac.load()
    torch.cuda.set_device(0)
    n = args.n
    case = W.single_vortex_case(n, eps=args.eps, tau=0.8, U=0.02, period_T=args.period)
    phi0 = W.circle(n, args.eps)
    if args.launch == "auto":
        launch = None
    elif args.launch:
        launch = tuple(int(v) for v in args.launch.split(","))
    else:
        default_case = args.n == 8192 and args.precision == "f32" and args.eps == 1.0 and args.period == 4096.0
        launch = profiled_launch() if default_case else None
        if launch is not None:
            print("bench: launch shape of the committed profiles: %s" % (launch,), file=sys.stderr, flush=True)
    print("bench: %dx%d %s, warmup %d, steps %d" % (n, n, args.precision, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    main_run = run_form(lbac, torch, case, phi0, args.precision, args.steps, args.warmup, launch=launch,
                        autotune=launch is None)
    nodes = n * n
    ms_per_step = main_run["ms_total"] / args.steps
    mlups = nodes * args.steps / (main_run["ms_total"] * 1e-3) / 1e6
    # the dominant kernel: the S-step launch, timed alone (HIP events on the
    # library's stream around the launches of the timed region that take S
    # steps).  It reads and writes the stored state once and takes spl steps.
    spl = main_run["steps_per_launch"]
    launch_ms = main_run["launch_ms"]
    updates_per_launch = nodes * spl
    # algorithmic HBM bytes of the method per launch: 72 B per node-update
    # (every population read and written once per step) x the node-updates of
    # one launch; the stored state itself crosses HBM once per launch
    alg_bytes = BYTES_PER_NODE_UPDATE * updates_per_launch
    state_bytes = main_run["bytes_per_node"] * nodes
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(main_run["launch"])
    valu = measured_valu_instructions(main_run["launch"])
    flops = measured_fp32_flops(main_run["launch"])
    valu_issue_frac = None if valu is None else valu / VALU_ISSUE_PER_S / (launch_ms * 1e-3)
    fp32_tflops = None if flops is None else flops / (launch_ms * 1e-3) / 1e12
    copy_gbs = state_bytes / (main_run["copy_us"] * 1e-6) / 1e9
    counter_gbs = None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9
    one_step = None
    if spl > 1 and args.one_step_steps > 0:
        # the same launch shape with the one-step kernel, for comparison
        print("bench: one-step kernel", file=sys.stderr, flush=True)
        lb = main_run["launch"]
        bx1 = lb[0] if lb[0] in (64, 128, 256) else 256  # tile widths the one-step kernel has
        r1 = run_form(lbac, torch, case, phi0, args.precision, args.one_step_steps, 0, launch=(bx1, lb[1], 2))
        ms1 = r1["ms_total"] / args.one_step_steps
        one_step = dict(launch=r1["launch"], steps=args.one_step_steps, ms_per_step=round(ms1, 4),
                        mlups=round(nodes / (ms1 * 1e-3) / 1e6, 1),
                        achieved_gbs=round(r1["bytes_per_node"] * nodes / (ms1 * 1e-3) / 1e9, 1))
    forms = {}
    for f in [s for s in args.forms.split(",") if s]:
        print("bench: form %s" % f, file=sys.stderr, flush=True)
        r = run_form(lbac, torch, case, phi0, f, args.steps, args.warmup, autotune=True)
        fm = nodes * args.steps / (r["ms_total"] * 1e-3) / 1e6
        forms[f] = dict(mlups=round(fm, 1), ms_per_step=round(r["ms_total"] / args.steps, 4),
                        hbm_gbs=round(r["bytes_per_node"] / r["steps_per_launch"] * nodes
                                      / (r["ms_total"] / args.steps * 1e-3) / 1e9, 1),
                        bytes_per_node=r["bytes_per_node"], e2=r["e2"], e1=r["e1"], mass_drift=r["mass_drift"],
                        e2_vs_plain=r["e2"] / main_run["e2"] if main_run["e2"] > 0 else None,
                        launch=r["launch"])
    batched = None
    if args.batch > 0:
        print("bench: batched form, %d instances" % args.batch, file=sys.stderr, flush=True)
        batched = batch_leg(lbac, torch, W, args.batch, 0, strip_h=args.batch_strip or None)
        if args.batch_f16:
            # the same list with shifted FP16 storage (the precision form inside the batched one)
            print("bench: batched form, FP16 shifted storage", file=sys.stderr, flush=True)
            b16 = batch_leg(lbac, torch, W, args.batch, 0, strip_h=args.batch_strip or None, seq_cap=0,
                            precision="f32_f16store")
            e2_32 = np.array(batched["e2_per_instance"])
            e2_16 = np.array(b16["e2_per_instance"])
            batched["f32_f16store"] = dict(mlups=b16["mlups"], ms=b16["ms"], strip_h=b16["strip_h"],
                                           bitwise_equal_probe=b16["bitwise_equal_probe"], e2_at_T=b16["e2_at_T"],
                                           e2_ratio_vs_f32_median=float(np.median(e2_16 / e2_32)),
                                           e2_ratio_vs_f32_max=float(np.max(e2_16 / e2_32)))
    closure = None
    if args.closure_steps > 0:
        print("bench: closure", file=sys.stderr, flush=True)
        closure = closure_leg(lbac, torch, case, phi0, args.closure_steps)
        closure["vs_plain_mlups"] = round(closure["mlups"] / mlups, 4)
    training = None
    if args.train_steps > 0:
        print("bench: closure training", file=sys.stderr, flush=True)
        training = train_leg(lbac, torch, args.train_steps)
    d3 = None
    c1 = None
    if args.c1_steps > 0:
        print("bench: 64^2 FP64, %d steps" % args.c1_steps, file=sys.stderr, flush=True)
        c1 = c1_leg(lbac, torch, W, args.c1_steps)
    c2 = None
    if args.c2_steps > 0:
        print("bench: 1024^2 storage forms, %d steps" % args.c2_steps, file=sys.stderr, flush=True)
        c2 = c2_leg(lbac, torch, W, 1024, args.c2_steps)
    if args.grid3d > 0:
        print("bench: 3-D form %d^3" % args.grid3d, file=sys.stderr, flush=True)
        launch3d = tuple(int(v) for v in args.launch3d.split(",")) if args.launch3d else None
        d3 = leg_3d(lbac, torch, W, args.grid3d, args.steps3d, launch=launch3d)
    cpu = None
    if args.cpu_steps > 0:
        print("bench: cpu baseline (%d oracle steps)" % args.cpu_steps, file=sys.stderr, flush=True)
        cpu = cpu_baseline(phi0, case, args.cpu_steps)
    line = {
        "metric": "MLUPS + HBM GB/s (% peak), D2Q9 phase-field step; L2 shape error at t=T",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32"}.get(args.precision, "f32"),
        "data": "synthetic",
        "config": {"workload": "single vortex %dx%d, eps=%g, tau=0.8, U=0.02, period T=%g steps, %s storage"
                               % (n, n, args.eps, args.period, args.precision),
                   "grid": n, "precision": args.precision, "launch": main_run["launch"]},
        "roofline": dict(
            ({"bound": "alu", "achieved": round(fp32_tflops, 2), "peak": round(FP32_PEAK_TFLOPS, 1),
              "unit": "TFLOP/s", "frac": round(fp32_tflops / FP32_PEAK_TFLOPS, 4)} if fp32_tflops is not None else
             {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(achieved / HBM_PEAK_GBS, 4)}),
            traffic=None if traffic is None else round(traffic, 0),
            kernel="stepS_kernel_lds<improved, %d, %d, FP32 storage>" % (main_run["launch"][0], spl),
            steps_per_launch=spl, launch_ms=round(launch_ms, 4), launches_timed=main_run["full_launches"],
            valu={"instructions_per_launch": valu,
                  "issue_frac": None if valu_issue_frac is None else round(valu_issue_frac, 4),
                  "fp32_flops_per_launch": flops,
                  "fp32_flops_per_node_update": None if flops is None else round(flops / updates_per_launch, 1)},
            hbm={"bytes_per_node_update": BYTES_PER_NODE_UPDATE, "algorithmic_bytes_per_launch": alg_bytes,
                 "achieved_gbs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                 "state_bytes_per_launch": state_bytes,
                 "counter_gbs": None if counter_gbs is None else round(counter_gbs, 1),
                 "counter_frac": None if counter_gbs is None else round(counter_gbs / HBM_PEAK_GBS, 4),
                 "pattern_copy_gbs": round(copy_gbs, 1)}),
        "one_step_kernel": one_step,
        "shape_error": {"t": main_run["t_end"], "e2": main_run["e2"], "e1": main_run["e1"],
                        "mass_drift": main_run["mass_drift"]},
        "wall_s": round(main_run["wall_s"], 3),
        "forms": forms,
        "batched": batched,
        "closure": closure,
        "closure_training": training,
        "c1_64": c1,
        "c2_1024": c2,
        "d3q19": d3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
