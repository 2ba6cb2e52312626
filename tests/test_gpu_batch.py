"""Batched form: many instances in one persistent launch, through the C ABI.

Each instance must be bitwise equal to the same instance advanced alone by
lbac_step with FP32 storage (whose parity against the oracle is tested in
test_gpu_parity.py); one instance is also checked against the oracle
directly.  The time-out path is forced from the host (waits that ask for a
step that never completes, with a short time-out), so every workgroup exits.
"""
import sys

import numpy as np
import pytest

from oracle import lib as O
from paper_2203_05230_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_cases():
    cases, phis, steps = [], [], []
    c = W.single_vortex_case(64, eps=1.0, tau=0.8, U=0.04, period_T=80.0)
    cases.append(c), phis.append(W.circle(64, 1.0)), steps.append(40)
    c = W.zalesak_case(128, eps=0.5, tau=0.7, rev_steps=4000)
    cases.append(c), phis.append(W.slotted_disk(128, 0.5)), steps.append(33)
    c = dict(nx=100, ny=70, eps=1.5, tau=0.9, delta=1e-10, vel="uniform", ux=0.03, uy=-0.02)
    cases.append(c), phis.append(W.circle(100, 1.5, R_frac=0.2, yc_frac=0.5)[:70]), steps.append(27)
    c = W.single_vortex_case(192, eps=2.0, tau=0.65, U=0.02, period_T=384.0)
    cases.append(c), phis.append(W.circle(192, 2.0)), steps.append(17)
    c = W.single_vortex_case(64, eps=1.0)
    cases.append(c), phis.append(W.circle(64, 1.0)), steps.append(0)
    c = dict(nx=130, ny=90, eps=1.0, tau=0.75, delta=1e-10, vel="vortex", U=0.03, period_T=200.0)
    cases.append(c), phis.append(W.circle(130, 1.0)[:90]), steps.append(25)
    return cases, phis, steps


def single(lb, case, phi0, n, precision="f32"):
    sim = lb.Simulation({**case, "precision": precision}, phi0)
    sim.step(n)
    out = sim.phi()
    sim.close()
    return out


def test_batch_bitwise_equals_single_instances(gpu_lib):
    say("case: batch of 6 mixed instances vs single-instance runs")
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases, phis)
    b.run(steps)
    masses = b.masses()
    for k, (c, p, n) in enumerate(zip(cases, phis, steps)):
        inst = b.instance(k)
        assert inst.time() == n
        ref = single(gpu_lib, c, p, n)
        assert np.array_equal(inst.phi(), ref), k
        assert np.array_equal(b.phi(k), ref), k  # lbac_batch_phi
        assert masses[k] == inst.mass(), k       # lbac_batch_mass
    b.close()


@pytest.mark.parametrize("precision", ["f32_f16store", "f32_bf16store"])
def test_batch_16bit_storage_bitwise_equals_single_instances(gpu_lib, precision):
    """Shifted 16-bit storage in the batch (FP32 between the steps of a pass,
    rounded once per pass): bitwise the single-instance form, over two runs
    (the second continues from the first's state) and two strip heights."""
    say("case: batch of 6 mixed instances,", precision)
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases, phis, precision=precision)
    b.run(steps)
    b.set_shape(24)
    b.run(steps)
    for k, (c, p, n) in enumerate(zip(cases, phis, steps)):
        inst = b.instance(k)
        assert inst.time() == 2 * n
        # 16-bit storage rounds once per launch, so the single run takes the
        # three-step launches and the same two calls (n // 3 three-step
        # launches, then n mod 3 one-step ones, each time)
        sim = gpu_lib.Simulation({**c, "precision": precision}, p)
        sim.set_launch(224, 40, 4)
        sim.step(n)
        sim.step(n)
        assert np.array_equal(inst.phi(), sim.phi()), k
        sim.close()
    b.close()


@pytest.mark.parametrize("precision", ["f32", "f32_f16store", "f32_bf16store"])
def test_batch_tiles_off_the_lines_bitwise(gpu_lib, precision):
    """Instances cut into 240-column tiles whose second tile starts off a
    128-byte line of the storage (x0 = 240: 960 bytes in FP32, 480 in 16-bit),
    so the tile function hands the head columns to its halo wavefront, and
    ragged last tiles of 20 to 160 columns; a 960-column instance also has
    16-bit tiles that start half a line and a quarter of a line in: bitwise
    the single runs."""
    say("case: batch tiles off the lines,", precision)
    shapes = [(500, 40, 10), (272, 33, 7), (400, 24, 12), (336, 50, 5), (960, 20, 5)]
    cases, phis, steps = [], [], []
    for i, (nx, ny, n) in enumerate(shapes):
        rng = np.random.default_rng(40 + i)
        phi = W.circle(max(nx, ny), 1.0, R_frac=0.3, yc_frac=0.5)[:ny, :nx] * 0.9 + 0.05 * rng.random((ny, nx))
        if i % 2:
            c = dict(nx=nx, ny=ny, eps=1.0, tau=0.8, delta=1e-10, vel="uniform", ux=0.03, uy=-0.021)
        else:
            c = dict(nx=nx, ny=ny, eps=1.0, tau=0.7, delta=1e-10, vel="vortex", U=0.03, period_T=100.0)
        cases.append(c), phis.append(np.ascontiguousarray(phi)), steps.append(n)
    b = gpu_lib.Batch(cases, phis, precision=precision)
    b.set_shape(16)
    b.run(steps)
    for k, (c, p, n) in enumerate(zip(cases, phis, steps)):
        sim = gpu_lib.Simulation({**c, "precision": precision}, p)
        sim.set_launch(224, 40, 4)
        sim.step(n)
        assert np.array_equal(b.instance(k).phi(), sim.phi()), (k, precision)
        sim.close()
    b.close()


@pytest.mark.parametrize("strip_h", [8, 9, 32, 64, 128])
def test_batch_shapes_and_continuation(gpu_lib, strip_h):
    say("case: batch strip height", strip_h)
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases, phis)
    b.set_shape(strip_h)
    first = [n // 2 for n in steps]
    b.run(first)
    b.run([n - f for n, f in zip(steps, first)])
    for k, (c, p, n) in enumerate(zip(cases, phis, steps)):
        assert np.array_equal(b.instance(k).phi(), single(gpu_lib, c, p, n)), k
    b.close()


def test_batch_autotune_keeps_state(gpu_lib):
    say("case: batch autotune")
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases, phis)
    b.run(steps)
    before = [b.instance(k).phi() for k in range(len(cases))]
    ms = b.autotune(4)
    assert ms > 0
    for k in range(len(cases)):
        assert np.array_equal(b.instance(k).phi(), before[k])
        assert b.instance(k).time() == steps[k]
    b.run([3] * len(cases))
    for k, (c, p, n) in enumerate(zip(cases, phis, steps)):
        assert np.array_equal(b.instance(k).phi(), single(gpu_lib, c, p, n + 3)), k
    b.close()


def test_batch_instance_matches_oracle(gpu_lib):
    say("case: batch instance vs oracle")
    n = 96
    case = W.single_vortex_case(n, eps=1.0, tau=0.8, U=0.03, period_T=600.0)
    phi0 = W.circle(n, 1.0)
    other = W.zalesak_case(128, eps=1.0, tau=0.9, rev_steps=4000)
    b = gpu_lib.Batch([case, other], [phi0, W.slotted_disk(128, 1.0)])
    b.run([300, 150])
    ref = O.run(O.Params(n, n, eps=1.0, tau=0.8, delta=1e-10, vel_kind=O.VEL_VORTEX, U=0.03, period_T=600.0),
                phi0, 300)
    got = b.instance(0).phi()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
    m = b.instance(1).mass()
    assert abs(m - W.slotted_disk(128, 1.0).sum()) / m < 1e-5
    b.close()


def test_batch_seeded_list_subset(gpu_lib):
    """Instances drawn by the seeded generator of the batched workload (sides
    128..512, eps in {0.5, 1, 2}, tau in [0.6, 1]; vortex and slotted disk),
    with the step counts cut short for the test."""
    say("case: seeded batch list, 12 instances")
    cases = W.batch_cases(count=12, seed=3)
    phis = [W.initial_field(c) for c in cases]
    steps = [min(c["steps"], 20 + 3 * k) for k, c in enumerate(cases)]
    b = gpu_lib.Batch(cases, phis)
    b.run(steps)
    for k in (0, 5, 6, 11):
        assert np.array_equal(b.instance(k).phi(), single(gpu_lib, cases[k], phis[k], steps[k])), k
    b.close()


def test_batch_benchmark_list_at_full_lengths(gpu_lib):
    """The benchmark's batched workload as timed: the 256 seeded instances
    (sides 128..512) over their whole runs (vortex 8 N, slotted disk 64 N
    steps; 1 024 to 32 768 steps), strips of 80 rows.  Every instance reaches
    its step count with its mass kept; the two longest runs, the two shortest
    and four between are bitwise equal to the same instances advanced alone."""
    say("case: benchmark batch list, 256 instances, full lengths")
    cases = W.batch_cases(count=256, seed=0)
    phis = [W.initial_field(c) for c in cases]
    steps = [c["steps"] for c in cases]
    b = gpu_lib.Batch(cases, phis)
    b.set_shape(80)
    b.run(steps)
    for k, (c, p0) in enumerate(zip(cases, phis)):
        inst = b.instance(k)
        assert inst.time() == steps[k], k
        m0 = float(p0.astype(np.float64).sum())
        assert abs(inst.mass() - m0) / m0 < 5e-5, k  # FP32 rounding over up to 32 768 steps
    order = sorted(range(256), key=lambda k: (steps[k] * cases[k]["nx"] * cases[k]["ny"], k))
    probe = order[:2] + order[-2:] + order[64:256:48]
    got = {k: b.instance(k).phi() for k in probe}
    b.close()
    for k in probe:
        say("  probe", k, cases[k]["nx"], steps[k])
        assert np.array_equal(got[k], single(gpu_lib, cases[k], phis[k], steps[k])), k


def oracle_params(c):
    if c["vel"] == "rotation":
        return O.Params(c["nx"], c["ny"], eps=c["eps"], tau=c["tau"], delta=c["delta"], vel_kind=O.VEL_ROTATION,
                        omega=c["omega"], cx=c["cx"], cy=c["cy"])
    return O.Params(c["nx"], c["ny"], eps=c["eps"], tau=c["tau"], delta=c["delta"], vel_kind=O.VEL_VORTEX,
                    U=c["U"], period_T=c["period_T"])


def test_batch_small_seeded_instances_match_oracle(gpu_lib):
    """Eight small instances from the batched workload's seeded generator
    (sides 32..96, both flows, eps and tau drawn as in the full list), each
    against the FP64 oracle after its own step count (FP32 storage: relative
    L2 <= 1e-5)."""
    say("case: 8 small seeded batch instances vs oracle")
    cases = W.batch_cases(count=8, seed=11, sides=(32, 48, 64, 96))
    phis = [W.initial_field(c) for c in cases]
    steps = [60 + 13 * k for k in range(8)]
    b = gpu_lib.Batch(cases, phis)
    b.run(steps)
    for k, c in enumerate(cases):
        ref = O.run(oracle_params(c), phis[k], steps[k])
        err = float(np.linalg.norm(b.instance(k).phi() - ref) / np.linalg.norm(ref))
        say("  instance %d (%s, n %d, eps %g, tau %.3f, %d steps): rel L2 %.2e" % (
            k, c["vel"], c["nx"], c["eps"], c["tau"], steps[k], err))
        assert err <= 1e-5, k
    b.close()


def test_batch_rejects_short_strips(gpu_lib):
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases[:2], phis[:2])
    with pytest.raises(gpu_lib.LbacError):
        b.set_shape(7)
    b.close()


def test_batch_stall_times_out_and_reports(gpu_lib):
    """Every wait asks for a step that never completes; with a 50 ms time-out
    every workgroup exits and the run reports a device error.  The passes that
    did run overwrote both buffers of some instances, so afterwards the batch
    and its instances refuse every call with LBAC_ESTATE."""
    say("case: batch forced stall")
    cases, phis, steps = mixed_cases()
    b = gpu_lib.Batch(cases, phis)
    b.set_timeout(0.05, test_stall=True)
    with pytest.raises(gpu_lib.LbacError) as ei:
        b.run([11] * len(cases))
    assert ei.value.code == gpu_lib.LBAC_EDEVICE
    b.set_timeout(20.0, test_stall=False)
    with pytest.raises(gpu_lib.LbacError) as ei:
        b.run([5] * len(cases))
    assert ei.value.code == gpu_lib.LBAC_ESTATE
    for call in (lambda i: i.phi(), lambda i: i.mass(), lambda i: i.step(1)):
        with pytest.raises(gpu_lib.LbacError) as ei:
            call(b.instance(0))
        assert ei.value.code == gpu_lib.LBAC_ESTATE
    b.close()
