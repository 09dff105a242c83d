"""CPU unit checks of the serving loop's host bookkeeping: the arena's first-fit allocator with
coalescing frees, and the removal of retired jobs from the active list on every way out of a
pass (normal end, error return, exception).  The checks are C++ (tests/arena_unit.cpp) built
with g++ against the library's own header."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2203_08680_amd", "csrc")


def test_arena_and_retire_bookkeeping(tmp_path):
    exe = str(tmp_path / "arena_unit")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror",
                    "-fsanitize=address,undefined", "-I", CSRC,
                    os.path.join(HERE, "arena_unit.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"
