"""The CPU oracle and the host planner built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only) and run over random inputs."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_check"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-Wall", "-Wextra"] + SAN +
                   ["-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "native", "oracle_check.c"),
                    os.path.join(ROOT, "oracle", "alnref.c"),
                    os.path.join(ROOT, "oracle", "foldref.c"), "-lpthread", "-o", str(exe)],
                   check=True)
    for seed in (1, 2):
        out = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=300)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr


def test_planner_under_sanitizers(tmp_path):
    """The planner (csrc/aln_api.cpp) compiled for the host with g++ and
    sanitizers, its kernel launchers replaced by stubs that report an error
    (a context without a device never launches), linked against the HIP
    runtime for the API it names."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "lib", "libamdhip64.so")):
        pytest.skip("HIP runtime library not found")
    exe = tmp_path / "planner_check"
    csrc = os.path.join(ROOT, "paper_2607_06225_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g"] + SAN +
                   ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                    "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(csrc, "aln_api.cpp"),
                    os.path.join(ROOT, "tests", "native", "launch_stubs.cpp"),
                    os.path.join(ROOT, "tests", "native", "planner_check.cpp"),
                    "-L", os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"),
                    "-lamdhip64", "-o", str(exe)], check=True, capture_output=True)
    for seed in (1, 2, 3):
        out = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=300)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr[-3000:]
