"""Host check of the GPU library's small dense linear algebra (Givens, LU,
Jacobi Hermitian eigensolver, Hessenberg-QR eigensolver), built with g++."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_dense_linear_algebra_on_host(tmp_path):
    exe = tmp_path / "linalg_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(ROOT, "tests", "linalg_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert "LINALG OK" in out.stdout
