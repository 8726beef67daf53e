"""Host code of the library under AddressSanitizer + UndefinedBehaviorSanitizer.

Every library source is compiled with the sanitizers on its host side only
(`-Xarch_host -fsanitize=...`; the device code is built unoptimised and never
launched) and linked into tests/host_checks.cpp, which drives the host-side
validation paths on the CPU: parameter checks over random and extreme shapes,
null handles and bad arguments of every entry point, status strings, and the
tuning-cache reader on valid, truncated and corrupted files.  No GPU is used
(HIP_VISIBLE_DEVICES is emptied).  Objects are cached under the package's
_build/sanitize keyed by a hash of the sources and flags.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1910_12979_amd")
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build", "sanitize")
DRIVER = os.path.join(ROOT, "tests", "host_checks.cpp")

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g", "-fPIC", "-std=c++17",
         "-ffp-contract=off", "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-Wno-unused-value",
         "-I", os.path.join(ROOT, "include"), *SAN]


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p if os.path.exists(p) else None


def _sources():
    from paper_1910_12979_amd.build import SOURCES
    return SOURCES


def _key() -> str:
    h = hashlib.sha1(" ".join(FLAGS).encode())
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))]
    files += [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))]
    files.append(DRIVER)
    for f in files:
        with open(f, "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def _build(hipcc: str) -> str:
    exe = os.path.join(OUT, "host_checks")
    stamp = os.path.join(OUT, "stamp")
    key = _key()
    if os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == key:
        return exe
    os.makedirs(OUT, exist_ok=True)

    def one(src):
        obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        r = subprocess.run([hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitizer build of {src} failed:\n{r.stderr[-4000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, _sources()))
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                        *SAN, "-I", os.path.join(ROOT, "include"), "-x", "c++", DRIVER, "-x", "none", *objs,
                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stderr[-4000:]}")
    with open(stamp, "w") as fh:
        fh.write(key)
    return exe


def test_host_paths_clean_under_asan_ubsan(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not installed")
    exe = _build(hipcc)
    env = dict(os.environ)
    env.update(HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="", MACPROJ_TUNE_CACHE="",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
