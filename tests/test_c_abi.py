"""include/sv.h compiles as plain C99 and links against libsv.so; a C program
drives the host-only entry points (no GPU needed)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_is_c99_and_links(tmp_path):
    exe = tmp_path / "abi_smoke"
    lib_dir = os.path.join(ROOT, "paper_2111_06868_amd")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic",
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c", "abi_smoke.c"),
                           "-L", lib_dir, "-l:libsv.so", "-Wl,-rpath," + lib_dir, "-lm",
                           "-o", str(exe)])
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=60)
    assert r.returncode == 0, r.stdout
    assert r.stdout.startswith("ok")
