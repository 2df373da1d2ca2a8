"""bench.py host-side behaviour (no GPU): the one-GPU contract and the helpers
that describe the measurement."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_kernel_precision_option_parses():
    # parsed before the GPU check: without a GPU the run stops there (exit 2)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--kernel-only",
                        "--kernel-precision", "f32", "--steps", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "needs a GPU" in r.stderr, r.stderr
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--kernel-only",
                        "--kernel-precision", "f16"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "invalid choice" in r.stderr


def test_host_cpu_and_source_digest():
    import bench
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["logical_cpus"] >= h["nproc"]
    assert isinstance(h["cpu_model"], str) and h["cpu_model"]
    d = bench.source_digest()
    assert len(d) == 16 and all(c in "0123456789abcdef" for c in d)
    assert d == bench.source_digest()
    # the digest covers the kernel, its device helpers and the launch settings
    assert [os.path.basename(p) for p in bench.STEP_SOURCES] == [
        "pond_step.hip", "pond_device.hpp", "pond_api.hip"]


def test_source_digest_ignores_comments_only(tmp_path):
    import bench
    code = 'int f(int x) { // twice\n  return 2 * x; /* block */ }\nconst char* s = "a // b";\n'
    a = tmp_path / "a.hip"
    a.write_text(code)
    b = tmp_path / "b.hip"
    b.write_text(code.replace("// twice", "// doubled").replace("/* block */", "") + "\n\n")
    c = tmp_path / "c.hip"
    c.write_text(code.replace("2 * x", "3 * x"))
    d = tmp_path / "d.hip"
    d.write_text(code.replace('"a // b"', '"a // c"'))
    assert bench.source_digest([str(a)]) == bench.source_digest([str(b)])
    assert bench.source_digest([str(a)]) != bench.source_digest([str(c)])
    assert bench.source_digest([str(a)]) != bench.source_digest([str(d)])


def test_flop_count_per_node_pass():
    import bench
    # 16 populations x 16 points x 42, 8 departure coordinates x 16, 7 x 16
    assert bench.FLOPS_PER_NODE_PASS == 10992
