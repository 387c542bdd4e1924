"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle: oracle.c built with gcc's sanitizers (and leak checking) and
  driven through every routine -- all four network modes, camera maps,
  detection, rounding, the split, FP8 storage, the gate's forward, BCE,
  backward and Adam -- by ``tests/sanitize/oracle_driver.c``.
* The library's host side: every HIP source rebuilt with the sanitizers on its
  host code only (``-Xarch_host`` before each flag; device code is unchanged),
  and ``tests/sanitize/abi_driver.c`` run against it: weights parsing over
  every truncation of a residual and of a dense-connection blob and a bad magic, config refusals before any
  device call, NULL handles, error text.  No GPU is needed (none is used).
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

import oracle
import smlm_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["address", "undefined"]


def _host_san_flags():
    out = []
    for s in SAN:
        out += ["-Xarch_host", f"-fsanitize={s}"]
    return out + ["-Xarch_host", "-fno-omit-frame-pointer"]


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-std=c99", "-g", "-O1", "-fopenmp", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
           "-fsanitize=" + ",".join(SAN), oracle._SRC, os.path.join(HERE, "oracle_driver.c"), "-o", str(exe), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "oracle driver ok" in r.stdout, r.stderr[-3000:]


def _clang_rt_dir():
    found = glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return os.path.dirname(found[0]) if found else None


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang")
def test_abi_host_paths_under_sanitizers(tmp_path):
    rt = _clang_rt_dir()
    if rt is None:
        pytest.skip("clang's ASan runtime is not installed")
    csrc = os.path.join(ROOT, "paper_2410_02314_amd", "csrc")
    base = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *_host_san_flags(),
            "-I", os.path.join(ROOT, "include"), "-I", csrc]

    def compile_one(src):
        obj = tmp_path / (os.path.basename(src)[:-4] + ".o")
        subprocess.check_call(base + ["-c", src, "-o", str(obj)], stderr=subprocess.DEVNULL)
        return str(obj)

    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, sorted(glob.glob(os.path.join(csrc, "*.hip")))))
    lib = tmp_path / "libdloc.so"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *_host_san_flags(), "-shared-libsan",
                           "-o", str(lib), *objs, "-Wl,-rpath,/opt/rocm/lib"], stderr=subprocess.DEVNULL)
    exe = tmp_path / "abi_driver"
    subprocess.check_call([CLANG, "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer", "-shared-libsan",
                           "-fsanitize=" + ",".join(SAN), "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "abi_driver.c"), "-o", str(exe), "-L", str(tmp_path), "-ldloc",
                           f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", f"-Wl,-rpath,{rt}"])
    # leaks are not checked here: the HIP runtime's own allocations would show
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    for name, seed in [("A", 1), ("D", 3)]:          # a residual (DLW1) and a dense (DLD1) blob
        spec, w = S.make_net(name, seed)
        blob = tmp_path / f"{name}.blob"
        blob.write_bytes(S.serialize_weights(spec, w))
        r = subprocess.run([str(exe), str(blob)], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0 and "abi driver ok" in r.stdout, (name, r.stderr[-3000:])
    shutil.rmtree(tmp_path, ignore_errors=True)
