"""Host-only check of the device-budget allocator behind the request server
(paper_2607_06225_amd/csrc/arena.h), built with g++ and fuzzed."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_fuzz(tmp_path):
    exe = tmp_path / "arena_fuzz"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra",
                    "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_2607_06225_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "arena_fuzz.cpp"), "-o", str(exe)],
                   check=True)
    for seed in (1, 2, 3):
        out = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
