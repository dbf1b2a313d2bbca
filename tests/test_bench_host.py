"""Host logic of the step bench: the update count per step and the
compulsory-byte model that the roofline line divides by the measured
launch time (no GPU needed)."""
import bench
import rte_inputs as ri


def test_stages_per_step_follow_the_scheme():
    # RK4 evaluates the operator four times per step, forward Euler once
    assert bench.stages_per_step("rk4") == 4
    assert bench.stages_per_step("euler") == 1
    assert bench.stages_per_step(ri.workload("p7_spheres", n=16).scheme) == 4
    assert bench.stages_per_step(ri.workload("paper_transient", n=16).scheme) == 1


def test_compulsory_bytes_of_the_128_p7_step():
    # F = 64 moments x 128^3 x 4 B; the fused inverse pass reads the coupled
    # spectrum, stage input and u (2.75F averaged over the stages), writes the
    # stage output and the next spectrum (2F), reads the 8 per-degree loss
    # maps and, in one stage of four, reads and writes the FP64 fluence
    n, N, M, s = 128, 7, 64, 4
    F = M * n ** 3 * s
    assert F == 536870912
    assert bench.algorithmic_bytes("zderiv", n, M, N, s) == 2 * F
    assert bench.algorithmic_bytes("couple", n, M, N, s) == 3 * F
    inv = bench.algorithmic_bytes("inv_plane", n, M, N, s)
    assert abs(inv - (4.75 * F + 8 * n ** 3 * 4 + 4 * n ** 3)) < 1
    assert abs(inv / 1e9 - 2.626) < 5e-4
    # per RK4 step: four stages of z derivative, coupling and fused plane pass
    step = 4 * (2 * F + 3 * F) + 4 * inv
    assert abs(step / 1e9 - 21.24) < 0.01
