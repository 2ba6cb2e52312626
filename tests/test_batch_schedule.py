"""The batched form's schedule, checked on the CPU (no GPU involved).

lbac_batch_schedule_check builds the items, dependency lists and pass-major
slot tables with the library's own host code and runs the kernel's slot
protocol (take the next slot number, wait for the previous pass of the
dependencies, work, publish) with a bounded number of workgroups running at
once and their actions interleaved at random.  The schedule must finish
without deadlock and without a read of a tile that does not hold the previous
pass or a write into a tile another running slot reads, whatever number of
workgroups the device keeps resident -- down to one.
"""
import numpy as np
import pytest

from paper_2203_05230_amd import lbac
from paper_2203_05230_amd import workloads as W


@pytest.mark.parametrize("workers", [1, 2, 7, 64, 512])
def test_benchmark_list_without_deadlock_at_any_residency(workers):
    """The 256-instance batched list (sides 128-512), 48 steps each (16 passes,
    the first launch of the benchmark's tuning), with 1 to 512 workgroups
    running at once."""
    cases = W.batch_cases(256, seed=0)
    shapes = [(c["nx"], c["ny"]) for c in cases]
    verdict, ran = lbac.batch_schedule_check(shapes, [48] * 256, 40, workers, seed=workers)
    assert verdict == 0, verdict
    strips = [max(1, min(int(ny / 40 + 0.5), ny // 8)) for _, ny in shapes]  # nearest count, balanced heights
    items_min = sum(-(-nx // 240) * s for (nx, _), s in zip(shapes, strips))
    items_max = sum(-(-nx // 16) * s for (nx, _), s in zip(shapes, strips))
    assert items_min * 16 <= ran <= items_max * 16 and ran % 16 == 0


@pytest.mark.parametrize("seed", range(6))
def test_uneven_lengths_ragged_grids_and_remainder_passes(seed):
    """Instances that retire at different passes (step counts that are not
    multiples of three, zero steps), ragged and tiny grids, several strip
    heights and residencies."""
    rng = np.random.default_rng(seed)
    shapes = [(int(a), int(b)) for a, b in zip(rng.integers(3, 300, 12), rng.integers(3, 300, 12))]
    shapes += [(1, 64), (64, 1), (5, 3), (224, 224), (225, 41), (240, 33), (496, 40), (512, 24)]
    nsteps = [int(v) for v in rng.integers(0, 40, len(shapes))]
    for strip_h in (8, 13, 40):
        for workers in (1, 3, 40):
            verdict, ran = lbac.batch_schedule_check(shapes, nsteps, strip_h, workers, seed=seed * 100 + workers)
            assert verdict == 0, (strip_h, workers, verdict)
            assert ran > 0


def test_full_length_schedule_of_a_reduced_list():
    """Real uneven retirement: vortex runs of 8 N steps and slotted disks of
    64 N steps on small sides, so that long runs continue alone for many
    passes after the short ones retired."""
    cases = W.batch_cases(16, seed=3, sides=(32, 48, 64), vortex_steps_per_side=8, rev_steps_per_side=64)
    shapes = [(c["nx"], c["ny"]) for c in cases]
    nsteps = [c["steps"] for c in cases]
    verdict, ran = lbac.batch_schedule_check(shapes, nsteps, 16, 24, seed=7)
    assert verdict == 0
    assert max(nsteps) > 3 * min(nsteps)


@pytest.mark.parametrize("nx,tiles", [(512, 3), (500, 3), (480, 2), (384, 2), (256, 2), (241, 2), (240, 1),
                                       (192, 1), (32, 1), (1000, 5)])
def test_column_tiles_of_an_instance(nx, tiles):
    """Column tiles of at most 240 columns in multiples of 16, chosen for the
    fewest wavefronts per row, then the fewest tiles: 480 columns take two
    tiles (three with 224-column tiles), 512 three (240 + 240 + 32).  One
    strip and 48 steps (16 full passes) run 16 slots per tile."""
    verdict, ran = lbac.batch_schedule_check([(nx, 40)], [48], 40, 4, seed=1)
    assert verdict == 0 and ran == 16 * tiles


def test_rejects_bad_sizes():
    with pytest.raises(lbac.LbacError):
        lbac.batch_schedule_check([(16, 16)], [3], 4, 1)  # strip below the minimum
    with pytest.raises(lbac.LbacError):
        lbac.batch_schedule_check([(0, 16)], [3], 16, 1)


@pytest.mark.parametrize("workers", [1, 7, 64, 512])
def test_fixed_item_lists_deadlock_when_not_all_resident(workers):
    """The earlier form of this schedule gave every workgroup a fixed list of
    items walked pass by pass; with fewer workgroups resident than lists (the
    check runs half of them), a resident workgroup waits for an item owned by
    one that never starts, and every resident one ends up waiting: the stall
    that form showed on a process's first batch launch.  The check must see
    it, at every residency."""
    cases = W.batch_cases(256, seed=0)
    shapes = [(c["nx"], c["ny"]) for c in cases]
    verdict, ran = lbac.batch_schedule_check(shapes, [48] * 256, 40, workers, seed=1, protocol=2)
    assert verdict == 1 and ran < 72368


@pytest.mark.parametrize("shapes", [[(64, 64)], [(96, 80), (64, 40)], [(300, 50)]])
def test_check_detects_hazards_without_the_waits(shapes):
    """Few items per pass and eight workgroups: without the dependency waits
    a pass starts before its neighbours published the previous one (the
    check reports the hazard); with them it never does."""
    for seed in range(5):
        assert lbac.batch_schedule_check(shapes, [30] * len(shapes), 16, 8, seed=seed, protocol=1)[0] == 2
        assert lbac.batch_schedule_check(shapes, [30] * len(shapes), 16, 8, seed=seed, protocol=0)[0] == 0
