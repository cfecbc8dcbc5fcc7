"""The benchmark's command-line contract on the CPU: more than one GPU is
refused with a message before anything touches a device, and the kernel
source hash that keys the stored HBM-traffic figures ignores comments."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_2512_18010_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "kernels.hip").write_text("int a; // one\n\nint b;\n")
    eng = "#include <x>\nnamespace scff {\nint c;\nstruct DeviceBuffer {};\nint runtime_decl();\n}\n"
    (csrc / "engine.h").write_text(eng)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    (csrc / "kernels.hip").write_text("int a; // a different comment\n// and a new one\nint b;   \n")
    assert bench.kernel_source_hash() == h0
    # engine.h outside the kernel's layout part (includes, runtime declarations) is not hashed
    (csrc / "engine.h").write_text(eng.replace("#include <x>", "#include <y>").replace("runtime_decl", "other"))
    assert bench.kernel_source_hash() == h0
    (csrc / "engine.h").write_text(eng.replace("int c;", "int c2;"))
    assert bench.kernel_source_hash() != h0
    (csrc / "engine.h").write_text(eng)
    (csrc / "kernels.hip").write_text("int a;\nint b2;\n")
    assert bench.kernel_source_hash() != h0


def test_roofline_picks_the_binding_pipe():
    """The roofline object names the pipe with the larger algorithmic time
    bound: the matrix cores for FP32 contraction with many transitions, the
    vector units when the split-BF16 contraction is cheap."""
    sys.path.insert(0, ROOT)
    import bench
    K, R, ns, nq = 59236, 234720, 24, 96 ** 3
    r = bench.grid_roofline(K, R, ns, nq, "fp32", 100.0)
    a = r["algorithmic"]
    assert r["bound"] == "mfma" and abs(a["t_mfma_ms"] - 4.0 * K * ns * nq / 157.3e12 * 1e3) < 1e-9
    assert abs(r["frac"] - a["t_mfma_ms"] / 100.0) < 1e-12
    r = bench.grid_roofline(K, R, ns, nq, "bf16x3", 50.0)
    a = r["algorithmic"]
    assert r["bound"] == "alu" and abs(r["frac"] - a["t_valu_ms"] / 50.0) < 1e-12
    assert abs(a["t_mfma_ms"] - 3 * 4.0 * K * ns * nq / 2.5166e15 * 1e3) < 1e-9
