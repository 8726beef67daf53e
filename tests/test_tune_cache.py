"""The autotuner's persistent cache (host side, no GPU): entries keyed by
architecture and level shape survive a save / clear / load round trip and a
fresh process reading MACPROJ_TUNE_CACHE; malformed files change nothing and
entries whose tile does not match their configuration index are skipped."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ARCH = "gfx950:test-arch"


@pytest.fixture()
def M():
    from paper_1910_12979_amd import macproj
    if not os.path.exists(macproj.LIB_PATH):
        from paper_1910_12979_amd import build
        build.build()
    macproj.lib()
    macproj.tune_cache_clear()
    yield macproj
    macproj.tune_cache_clear()


def test_round_trip(M, tmp_path):
    path = tmp_path / "tune.json"
    M.tune_record((256, 256, 256), 11, rho=True, fp64=True, arch=ARCH)
    M.tune_record((128, 128, 128), 6, rho=True, fp64=False, arch=ARCH)
    M.tune_record((64, 64, 64), 12, rho=False, fp64=True, coarse=True, arch=ARCH)
    M.tune_record((64, 64, 64), 7, rho=False, fp64=True, coarse=False, arch="gfx942:other")
    assert M.tune_cache_save(str(path)) == 4
    doc = json.loads(path.read_text())
    assert doc["format"] == "macproj-sweep-tune-1" and len(doc["entries"]) == 4
    e = [x for x in doc["entries"] if x["n"] == [256, 256, 256]][0]
    assert e == {"arch": ARCH, "n": [256, 256, 256], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 11,
                 "tile": [64, 16, 64]}
    M.tune_cache_clear()
    assert M.tune_lookup((256, 256, 256), arch=ARCH) == -1
    assert M.tune_cache_load(str(path)) == 4
    assert M.tune_lookup((256, 256, 256), rho=True, fp64=True, arch=ARCH) == 11
    assert M.tune_lookup((128, 128, 128), rho=True, fp64=False, arch=ARCH) == 6
    assert M.tune_lookup((128, 128, 128), rho=True, fp64=True, arch=ARCH) == -1     # other precision
    assert M.tune_lookup((64, 64, 64), rho=False, coarse=True, arch=ARCH) == 12
    assert M.tune_lookup((64, 64, 64), rho=False, coarse=False, arch=ARCH) == -1    # other arch only
    assert M.tune_lookup((64, 64, 64), rho=False, coarse=False, arch="gfx942:other") == 7


def test_bad_files_and_entries(M, tmp_path):
    M.tune_record((256, 256, 256), 11, arch=ARCH)
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "macproj-sweep-tune-1", "entries": [{"arch": ')
    with pytest.raises(M.MGError):
        M.tune_cache_load(str(bad))
    other = tmp_path / "other.json"
    other.write_text('{"format": "something-else", "entries": []}')
    with pytest.raises(M.MGError):
        M.tune_cache_load(str(other))
    with pytest.raises(M.MGError):
        M.tune_cache_load(str(tmp_path / "missing.json"))
    assert M.tune_lookup((256, 256, 256), arch=ARCH) == 11          # unchanged by the failed loads
    mixed = tmp_path / "mixed.json"
    mixed.write_text("""{"format": "macproj-sweep-tune-1", "note": {"x": [1, "a]"]}, "entries": [
      {"arch": "%(a)s", "n": [96, 96, 96], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 0, "tile": [32, 8, 32]},
      {"arch": "%(a)s", "n": [48, 48, 48], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 0, "tile": [64, 16, 64]},
      {"arch": "%(a)s", "n": [16, 16, 16], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 2, "tile": [64, 8, 32]},
      {"arch": "%(a)s", "n": [64, 64, 64], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 99, "tile": [32, 8, 32]},
      {"arch": "%(a)s", "n": [32, 32, 32], "rho": 1, "fp64": 1, "coarse": 0, "cfg": 7, "tile": [32, 8, 8],
       "extra": [true, null, {"k": "v"}]}]}""" % {"a": ARCH})
    assert M.tune_cache_load(str(mixed)) == 2           # tile mismatch, a tile wider than the box, bad index
    assert M.tune_lookup((96, 96, 96), arch=ARCH) == 0
    assert M.tune_lookup((48, 48, 48), arch=ARCH) == -1
    assert M.tune_lookup((16, 16, 16), arch=ARCH) == -1
    assert M.tune_lookup((32, 32, 32), arch=ARCH) == 7
    with pytest.raises(M.MGError):
        M.tune_record((16, 16, 16), 2, arch=ARCH)          # 64-wide tile on a 16-wide level
    with pytest.raises(M.MGError):
        M.tune_record((64, 64, 64), 14, arch=ARCH)


def test_environment_file_is_read_by_a_fresh_process(M, tmp_path):
    path = tmp_path / "env.json"
    M.tune_record((128, 128, 64), 2, arch=ARCH)
    M.tune_cache_save(str(path))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1910_12979_amd import macproj as M\n"
            "print(M.tune_lookup((128, 128, 64), arch=%r))\n") % (ROOT, ARCH)
    env = dict(os.environ, MACPROJ_TUNE_CACHE=str(path), HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "2"
