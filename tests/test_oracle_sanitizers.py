"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(both of its precisions) and driven through every entry point on small
inputs, including an invalid theta and a singular R: no memory error, no
undefined behaviour, every call returns."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    src = os.path.join(ROOT, "oracle", "gp_oracle.c")
    objs = []
    flags = ["-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
    for real, sfx in (("double", "f64"), ("long double", "f80")):
        obj = str(tmp_path / f"o_{sfx}.o")
        subprocess.check_call(["gcc"] + flags + ["-c", src, "-o", obj, f"-DREAL={real}",
                                                 f"-DSFX(name)=name##_{sfx}"])
        objs.append(obj)
    exe = str(tmp_path / "drv")
    subprocess.check_call(["gcc"] + flags + [os.path.join(ROOT, "tests", "oracle_asan_driver.c")]
                          + objs + ["-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
