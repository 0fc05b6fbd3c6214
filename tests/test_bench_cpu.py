"""CPU checks of the benchmark's byte model and its command line (no GPU).

The roofline of the fused stage divides the method's algorithmic bytes by the
measured stage time.  Those bytes follow the FR data a stage must move: the state
(five state-sized streams), the two neighbour exchanges (five flux-point-sized
streams) and, on curved elements, the FP64 metrics.  Per DOF-update (one DOF through
the four stages of an RK4 step) they come to the figures of the scope table for
3D p = 3: 200 B (FP32, affine), 278 B (FP32, curved), 400 and 478 B in FP64, and
323 B / 252 B for curved p = 2 / p = 4 in FP32.
"""
import subprocess
import sys

import pytest

import bench


@pytest.mark.parametrize("order,real,curved,expect", [
    (3, 4, False, 200.0), (3, 4, True, 278.4), (3, 8, False, 400.0), (3, 8, True, 478.4),
    (2, 4, True, 323.2), (4, 4, True, 251.5)])
def test_algorithmic_bytes_per_dof_update(order, real, curved, expect):
    n = order + 1
    per_stage = bench.algorithmic_bytes_per_element_stage(3, order, real, curved)
    per_dof_update = 4 * per_stage / (n ** 3 * 5)
    assert abs(per_dof_update - expect) < 0.05, per_dof_update


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_counter_traffic_is_tied_to_the_variant_it_was_taken_on():
    """The committed batch counters cover the gather exchange on column metrics (variant mask
    417) with the default tiles, the second launch's half tile and the matrix-core first
    launch; any other variant reports no counter traffic."""
    assert bench.stage_kernel_name("k_stage_a", 417) == "k_stage_a<float, 3, 3, 3, 0, false>"
    assert bench.stage_kernel_name("k_stage_b", 417 | (2 << 11)) == "k_stage_b<float, 3, 3, 0, 3, 2, false>"
    assert bench.stage_kernel_name("k_stage_a", 417 | (1 << 13)) == "k_stage_a<float, 3, 3, 3, 0, true>"
    assert bench.stage_kernel_name("k_stage_b", 1 | (1 << 6)) == "k_stage_b<float, 3, 3, 0, 1, 0, false>"
    for kernel in ("k_stage_a", "k_stage_b"):
        t = bench.counters_traffic("batch", kernel, 417)
        if t is None:
            pytest.skip("the committed counters were taken on another kernel source")
        assert t > 0
        assert bench.counters_traffic("batch", kernel, 417 | (1 << 13)) is None
        assert bench.counters_traffic("batch", kernel, 417 | (2 << 9) | (2 << 11)) is None
    # the second launch's half tile and the matrix-core first launch have entries of their own
    b1 = bench.counters_traffic("batch", "k_stage_b", 417 | (1 << 11))
    a3 = bench.counters_traffic("batch", "k_stage_a", 417 | (3 << 9))
    assert b1 and a3 and b1 != bench.counters_traffic("batch", "k_stage_b", 417)
