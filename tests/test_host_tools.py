"""Host-side tools, on the CPU: bench.py's one-GPU contract, and the counter
bookkeeping (record_traffic's kernel names, source lists and per-dispatch
means; bench.py withholding a counter figure once the kernel's sources
changed)."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1111_2142_amd import record_traffic as rt  # noqa: E402


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_kernel_key_normalises_demangled_names():
    name = ("void lwacm::(anonymous namespace)::k_fwd_march_rolled<float, 128, false, false, "
            "false, 0, false, true>(lwacm::ProblemArgs, float const*, float*, unsigned int "
            "const*, HIP_vector_type<float, 4u> const*, lwacm::ReduceArgs)")
    assert rt.kernel_key(name) == "k_fwd_march_rolled<float,128,false,false,false,0,false,true>"
    assert rt.kernel_key("void lwacm::(anonymous namespace)::k_wall_correction<float>(x)") == \
        "k_wall_correction<float>"
    assert rt.kernel_key("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_sources_of_follows_local_includes():
    files = rt.sources_of("csrc/lwacm_march2.hip")
    assert files[0] == "csrc/lwacm_march2.hip"
    for f in ("csrc/lwacm_march_common.hpp", "csrc/lwacm_device.hpp"):
        assert f in files
    assert len(files) == len(set(files))
    for base, src in rt.KERNEL_SOURCE.items():
        assert os.path.exists(os.path.join(rt.PKG, src)), base


def test_mean_counter_averages_per_dispatch(tmp_path):
    p = tmp_path / "c.csv"
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    # two dispatches of one kernel, the first reported in two rows (summed)
    rows += ["1,void k_a<1>(int),FETCH_SIZE,10", "1,void k_a<1>(int),FETCH_SIZE,5",
             "2,void k_a<1>(int),FETCH_SIZE,25", "3,void k_b(int),FETCH_SIZE,1000",
             "3,void k_b(int),WRITE_SIZE,7"]
    p.write_text("\n".join(rows) + "\n")
    mean, n = rt.mean_counter(str(p), "FETCH_SIZE", "k_a<1>")
    assert (mean, n) == (20.0, 2)
    assert rt.largest_kernel(str(p), "FETCH_SIZE") == "k_b"


def test_bench_withholds_a_figure_once_the_sources_change(tmp_path):
    bench = _bench_module()
    pkg = tmp_path / "paper_1111_2142_amd"
    (pkg / "csrc").mkdir(parents=True)
    src = pkg / "csrc" / "k.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    rec = {"k_x<1>": {"sources": ["csrc/k.hip"], "sources_sha256": digest,
                      "hbm_bytes_per_launch": 1234, "valu_insts_per_launch": 99}}
    (pkg / "measured_traffic.json").write_text(json.dumps(rec))
    bench.ROOT = str(tmp_path)
    assert bench._measured_traffic("k_x<1>") == 1234
    assert bench._measured("k_x<1>", "valu_insts_per_launch") == 99
    assert bench._measured_traffic("k_y<1>") is None
    src.write_text("kernel source, changed\n")
    assert bench._measured_traffic("k_x<1>") is None


def test_committed_records_name_existing_sources():
    db = json.load(open(os.path.join(rt.PKG, "measured_traffic.json")))
    assert db
    for key, rec in db.items():
        assert key.split("<")[0] in rt.KERNEL_SOURCE, key
        for f in rec["sources"]:
            assert os.path.exists(os.path.join(rt.PKG, f)), (key, f)
        assert rec["hbm_bytes_per_launch"] > 0 and rec["fetch_scale"] > 0
