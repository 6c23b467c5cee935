"""The C ABI library on the CPU: it loads, exports every entry point the
header declares, and its host-side geometry logic (canonical hash, face
neighbours for the exchange operator, argument checks) works without a GPU.
No compute call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tilemag.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def tmg():
    from paper_2107_05364_amd import tilemag

    tilemag.load()
    return tilemag


def test_header_declares_the_abi():
    names = _declared()
    for must in ("tm_init", "tm_tensor_assemble", "tm_demag", "tm_run", "tm_server_submit"):
        assert must in names


def test_library_exports_every_declared_symbol(tmg):
    L = tmg.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header(tmg):
    assert sorted(tmg.EXPORTS) == _declared()
    for name in tmg.EXPORTS:
        assert callable(getattr(tmg, name)), name


def test_binding_constants_match_the_header(tmg):
    """Every TM_* enumerator the header assigns a value has the same value in
    the binding (layouts, precisions, integrators, status codes)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    pairs = re.findall(r"\b(TM_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)
    pairs += re.findall(r"#define\s+(TM_[A-Z0-9_]+)\s+\((-?\d+)\)", text)
    assert len(pairs) >= 15
    for name, val in pairs:
        if hasattr(tmg, name):
            assert getattr(tmg, name) == int(val), (name, val)
    for must in ("TM_LAYOUT_PSYM4", "TM_LAYOUT_PSYM6", "TM_PREC_BF16X3", "TM_DP45", "TM_EINVAL"):
        assert hasattr(tmg, must), must


def test_version_and_error_text(tmg):
    assert tmg.load().tm_version() >= 100
    with pytest.raises(tmg.TilemagError) as ei:
        tmg.tm_geometry_create(None, np.zeros((1, 3)), np.array([[1e-9, 0.0, 1e-9]]))
    assert ei.value.status == tmg.TM_EINVAL and "edge" in str(ei.value)
    with pytest.raises(tmg.TilemagError):
        tmg.tm_geometry_create(None, np.array([[np.nan, 0, 0]]), np.full((1, 3), 1e-9))


def test_geometry_hash_is_canonical(tmg):
    from paper_2107_05364_amd.workloads import grid

    c, s = grid(5, 4, 2, 5e-9, 5e-9, 3e-9)
    g1 = tmg.Geometry(None, c, s)
    g2 = tmg.Geometry(None, c.copy(), s.copy())
    c0 = c.copy()
    c0[0, 0] = -0.0 if c0[0, 0] == 0.0 else c0[0, 0]
    assert g1.hash == g2.hash
    c3 = c.copy()
    c3[3, 1] = np.nextafter(c3[3, 1], 1.0)
    assert tmg.Geometry(None, c3, s).hash != g1.hash
    s3 = s.copy()
    s3[7, 2] *= 1.0 + 2e-16
    assert tmg.Geometry(None, c, s3).hash != g1.hash


@pytest.mark.parametrize("which", ["grid", "film", "refined"])
def test_face_neighbours_match_oracle(tmg, orc, which):
    from paper_2107_05364_amd import workloads as W

    if which == "grid":
        c, s = W.grid(7, 3, 4, 5e-9, 4e-9, 3e-9)
    elif which == "film":
        wl = W.thin_film()
        c, s = wl.centers, wl.sizes
    else:
        wl = W.refined_slab(n_target=1500, lx=300e-9, ly=80e-9, lz=20e-9)
        c, s = wl.centers, wl.sizes
    g = tmg.Geometry(None, c, s)
    fa, fb, area, dist = orc.faces(c, s)
    assert g.nfaces == fa.shape[0]


def test_init_without_gpu_fails_cleanly(tmg):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = C.c_void_p()
    st = tmg.load().tm_init(0, C.byref(out))
    assert st in (tmg.TM_EDEVICE, tmg.TM_EINVAL)
    assert tmg.last_error()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; a request for more exits with a message
    (before touching any device)."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_tune_cache_file_round_trip(tmg, tmp_path):
    """The autotuner table's JSON file: entries load, save and load back
    unchanged; a missing file and a foreign or malformed one are refused
    (host logic only, no device)."""
    src = tmp_path / "tune.json"
    src.write_text(
        '{"tilemag_tune_cache": 1, "entries": [\n'
        ' {"arch": "gfx950:sramecc+:xnack-", "cus": 256, "layout": 4, "prec": 0, "n": 2500, "batch": 1, '
        '"choice": 1, "ms": 0.0127},\n'
        ' {"arch": "gfx950:sramecc+:xnack-", "cus": 256, "layout": 0, "prec": 0, "n": 512, "batch": 1, '
        '"choice": 10, "ms": 0.00426}\n]}\n')
    tmg.tm_tune_cache_clear()
    assert tmg.tm_tune_cache_size() == 0
    assert tmg.tm_tune_cache_load(str(src)) == tmg.TM_OK
    assert tmg.tm_tune_cache_size() == 2
    out = tmp_path / "out.json"
    tmg.tm_tune_cache_save(str(out))
    tmg.tm_tune_cache_clear()
    assert tmg.tm_tune_cache_load(str(out)) == tmg.TM_OK and tmg.tm_tune_cache_size() == 2
    again = tmp_path / "again.json"
    tmg.tm_tune_cache_save(str(again))
    assert again.read_text() == out.read_text()
    assert '"n": 2500, "batch": 1, "choice": 1, "ms": 0.0127' in out.read_text()
    assert tmg.tm_tune_cache_load(str(tmp_path / "missing.json")) == tmg.TM_ENOTFOUND
    bad = tmp_path / "bad.json"
    bad.write_text('{"something_else": 1}\n')
    with pytest.raises(tmg.TilemagError):
        tmg.tm_tune_cache_load(str(bad))
    bad.write_text('{"tilemag_tune_cache": 1, "entries": [\n {"arch": "gfx950", "cus": 256}\n]}\n')
    with pytest.raises(tmg.TilemagError):
        tmg.tm_tune_cache_load(str(bad))
    assert tmg.tm_tune_cache_size() == 2  # a refused file adds nothing
    tmg.tm_tune_cache_clear()
