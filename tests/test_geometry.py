"""Host check of the GPU library's site order and neighbour tables (bounds,
bijection, neighbours, colouring, XCD remap), compiled and run on the CPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_geometry_tables_on_host(tmp_path):
    exe = tmp_path / "geometry_check"
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", os.path.join(ROOT, "tests", "geometry_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert "GEOMETRY OK" in out.stdout
