"""CPU checks of the bench.py contract that need no GPU: the multi-GPU refusal and
the byte model of the PM step."""
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_step_bytes_add_up():
    # the per-stage algorithmic bytes of one PM step sum to b_alg_step: deposit, z and
    # y forward, the x pass, the y pass of the x component, the paired y pass, three
    # z inverse passes (one per component), and the gather
    for np_side, nm in ((256, 512), (256, 768), (512, 1024), (32, 64)):
        sb = bench.stage_bytes(np_side, nm)
        total = (sb["deposit"] + sb["fft_z_fwd"] + sb["fft_y_fwd"] + sb["fft_x_poisson"] + sb["fft_y_inv"]
                 + sb["fft_y_inv_pair"] + 3 * sb["fft_z_inv"] + sb["gather_kick_drift"])
        assert total == bench.b_alg_step(np_side, nm)
        # three independent inverse chains would move 16 C more
        c = nm * nm * (nm // 2 + 1)
        assert bench.b_alg_three_chains(np_side, nm) - bench.b_alg_step(np_side, nm) == 16 * c


def test_committed_profiles_cover_the_current_sources():
    # the roofline's traffic and rocprofv3 mean come from the committed summaries only
    # when those were taken on the current kernel sources, for the benchmarked bin depth
    traffic = bench.read_traffic("gather_kick_drift", "c1")
    prof = bench.read_profile_avg("gather_kick_drift", "c1", 32)
    assert traffic is not None and traffic > bench.stage_bytes(256, 512)["gather_kick_drift"]
    assert prof is not None and prof["kernel"] == "k_gather_sorted<32, 1>" and 0.1 < prof["avg_ms"] < 10
    assert bench.read_profile_avg("gather_kick_drift", "c1", 64) is None
    assert bench.read_profile_avg("no_such_stage", "c1", 32) is None
