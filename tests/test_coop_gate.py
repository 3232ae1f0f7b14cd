"""The process-wide gate that keeps at most one cooperative launch in flight
(paper_1303_1379_amd/csrc/mcm_gate.h), exercised on the CPU with threads
standing in for the library's callers: distinct owners never overlap, one
owner (a server's stream) may hold several launches, and a waiting caller
is not starved by a server that keeps launching.  No GPU involved."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1303_1379_amd", "csrc")


def test_coop_gate_threads(tmp_path):
    exe = str(tmp_path / "coop_gate_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I" + CSRC, "-o", exe,
                    os.path.join(HERE, "coop_gate_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
