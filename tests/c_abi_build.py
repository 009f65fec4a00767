"""Build helper for the plain C consumer of the library (tests/cpp/abi_c.c)."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "abi_c.c")
INC = os.path.join(ROOT, "include")
LIBDIR = os.path.join(ROOT, "paper_2011_00287_amd", "lib")


def compile_c_consumer(out_dir: str) -> str:
    """gcc -std=c11 -Wall -Werror against the public header, linked to the built library."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler")
    exe = os.path.join(out_dir, "abi_c")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-I" + INC, SRC, "-o", exe, "-L" + LIBDIR,
           "-llbchiral", "-Wl,-rpath," + LIBDIR, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C consumer failed to build:\n" + r.stdout + r.stderr)
    return exe
