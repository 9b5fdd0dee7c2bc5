"""Host-side logic of bench.py and the counter summaries (no GPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_summaries_parse_and_gate_on_source():
    from paper_2609_29554_amd import pmc
    sys.path.insert(0, ROOT)
    import bench
    names = ("pmc_traffic_lu_qd2048_lotkin_b128.md", "pmc_traffic_lu_qd2048_lotkin_b256.md",
             "pmc_traffic_gemm_td4096_int8.md", "pmc_traffic_limb_schur_p4096.md")
    for name in names:
        s = pmc.load(os.path.join(ROOT, "profiles", name))
        assert s is not None and s["kernels"]
        assert 1.5 < s["fetch_factor"] < 2.5 and 0.5 < s["write_factor"] < 1.5
        stage = "consumer"
        fams = [f for f in bench.STAGE_KERNELS[stage] if f in s["kernels"]]
        assert fams, name
        fam = fams[0]
        t = bench.traffic_of(stage, name)
        if s["kernel_source_sha256"] == pmc.source_sha():
            assert abs(t - s["kernels"][fam]["hbm_bytes_per_launch"]) <= 1e-9 * t and t > 0
        else:
            assert t is None     # measured on other kernel sources: not reported


def test_kernel_names_in_summaries():
    from paper_2609_29554_amd import pmc
    assert pmc.short_name("void (anonymous namespace)::k_gemm_i8_p<2, 4, 4>(signed char const*, "
                          "int)") == "k_gemm_i8_p<2, 4, 4>"
    assert pmc._family("(anonymous namespace)::k_limb_sub(unsigned long*, int*)") == "k_limb_sub"
    assert pmc._family("__amd_rocclr_copyBuffer") is None
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.endswith("_kernel_trace.md"):
            text = open(os.path.join(ROOT, "profiles", name)).read()
            assert "| `` |" not in text and "rocprofv3 --kernel-trace" in text


def test_gpu_count_guard():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_schur_shapes_and_op_counts():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.schur_shapes(2048, 256) == [(1792 - 256 * i, 256) for i in range(7)]
    assert bench.schur_shapes(100, 32)[-1] == (4, 32)
    P, U = bench.op_counts(512, 128)
    assert P > 0 and U > 0
