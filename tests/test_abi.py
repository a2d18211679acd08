"""The C-ABI library: it loads, exports every declared entry point, and its
host-side geometry matches the oracle's decomposition (no GPU needed)."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import schwarz
from paper_1508_02977_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(api.LIB_PATH):
        from paper_1508_02977_amd import build
        build.build()


def test_header_symbols_exported():
    _ensure_built()
    hdr = open(os.path.join(ROOT, "include", "sfdd.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sf_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", api.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT\s+(sf_\w+)", out))
    assert declared <= exported, declared - exported
    assert declared == set(api.exported_symbols())
    L = api.lib()
    for name in declared:
        assert getattr(L, name) is not None


def test_status_strings():
    _ensure_built()
    for code in (0, -1, -2, -3, -4, -5, 1, 2, 3):
        assert api.sf_status_string(code) not in ("unknown status", "")


@pytest.mark.parametrize("W,H,px,py,d", [(64, 64, 2, 2, 4), (640, 480, 4, 4, 8), (37, 29, 3, 2, 5),
                                         (23, 41, 2, 3, 6), (50, 9, 5, 1, 3), (1920, 1080, 12, 7, 8)])
def test_plan_matches_oracle_decomposition(W, H, px, py, d):
    _ensure_built()
    plan = api.sf_plan(W, H, 1, px, py, d)
    subs = schwarz.decompose(W, H, px, py, d)
    assert len(plan) == len(subs)
    for g, s in zip(plan, subs):
        assert g["box"] == (s.box[0], s.box[1], s.box[2], s.box[3])
        assert g["own"] == s.own
        assert g["cols"] == s.cols


def test_plan_batch_and_invalid():
    _ensure_built()
    plan = api.sf_plan(20, 10, 3, 2, 1, 2)
    assert [g["pair"] for g in plan] == [0, 0, 1, 1, 2, 2]
    with pytest.raises(api.SfError):
        api.sf_plan(1, 10, 1, 1, 1, 0)
    with pytest.raises(api.SfError):
        api.sf_plan(10, 10, 1, 11, 1, 0)


@pytest.mark.parametrize("W,H,n", [(48, 48, 12), (640, 480, 16), (1920, 1080, 84), (37, 29, 6), (64, 64, 7),
                                   (300, 136, 2), (5, 40, 8)])
def test_split_chooser_matches_oracle(W, H, n):
    from oracle import variants
    _ensure_built()
    assert api.sf_choose_split(W, H, n) == variants.choose_split(W, H, n)


def test_split_chooser_worked_example_and_invalid():
    # the paper's printed example (tests/golden/split_ratio_48x48.txt): the
    # chosen split has the largest printed ratio
    _ensure_built()
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "split_ratio_48x48.txt")
    rows = [tuple(line.split()) for line in open(golden) if line.strip() and not line.startswith("#")]
    best = max(float(r) for _, _, r in rows)
    px, py, r = api.sf_choose_split(48, 48, 12)
    assert (str(px), str(py), f"{best:g}") in rows and math.floor(r * 1000) / 1000 == best
    with pytest.raises(api.SfError):
        api.sf_choose_split(3, 3, 16)        # no split with at most one part per pixel
    with pytest.raises(api.SfError):
        api.sf_choose_split(48, 48, 0)


def test_sigma_bounds():
    _ensure_built()
    cfg_ok = api.make_config(32, 32, 1, 2, 2, 4, sigma=api.SF_SIGMA_MAX)
    cfg_bad = api.make_config(32, 32, 1, 2, 2, 4, sigma=api.SF_SIGMA_MAX + 0.5)
    assert api.lib().sf_plan(cfg_ok, None) == 4
    assert api.lib().sf_plan(cfg_bad, None) == api.SF_ERR_INVALID
    assert api.lib().sf_plan(api.make_config(32, 32, 1, 2, 2, 4, sigma=-1.0), None) == api.SF_ERR_INVALID


@pytest.mark.parametrize("W,H,px,py,d", [(64, 64, 2, 2, 4), (640, 480, 4, 4, 8), (1920, 1080, 12, 7, 8)])
def test_memory_bytes_linear_in_batch_and_tile_storage(W, H, px, py, d):
    _ensure_built()
    b1, b2, b5 = (api.sf_memory_bytes(W, H, b, px, py, d) for b in (1, 2, 5))
    # every pair repeats the same subdomains and fields; the factor workspace
    # is shared by chunks of at most 64 subdomains, so the bytes grow by the
    # same amount per pair once a batch has 64 subdomains, and never faster
    assert b5 - b1 <= 4 * (b2 - b1) and b2 > b1 > 0
    nsub = len(api.sf_plan(W, H, 1, px, py, d))
    k = -(-64 // nsub)
    bk, bk1, bk4 = (api.sf_memory_bytes(W, H, b, px, py, d) for b in (k, k + 1, k + 4))
    assert bk4 - bk == 4 * (bk1 - bk) > 0
    # FP32 tiles halve exactly the inverse Schur tiles: per subdomain, lines x
    # lower tiles of the padded line matrix (32x32 tiles), from the geometry alone
    tile_bytes = 0
    for g in api.sf_plan(W, H, 1, px, py, d):
        x0, x1, y0, y1 = g["box"]
        ms, nt = (y1 - y0, x1 - x0) if g["cols"] else (x1 - x0, y1 - y0)
        NT = -(-3 * ms // 32)
        tile_bytes += nt * NT * (NT + 1) // 2 * 32 * 32 * 8
    f32 = api.sf_memory_bytes(W, H, 1, px, py, d, factor_precision=api.SF_FP32)
    assert b1 - f32 == tile_bytes // 2
    assert b1 > tile_bytes


def test_memory_bytes_invalid():
    _ensure_built()
    with pytest.raises(api.SfError):
        api.sf_memory_bytes(0, 10)
    with pytest.raises(api.SfError):
        api.sf_memory_bytes(260, 257)          # lines of 257 nodes: above the largest line matrix (768)
    assert api.sf_memory_bytes(264, 256) > 0    # lines of 256 nodes: the largest


def test_library_built_from_the_current_sources():
    # the binding refuses a library whose embedded source digest differs from
    # the sources in the tree; the loaded one must match
    _ensure_built()
    from paper_1508_02977_amd import build
    assert api.lib().sf_build_digest().decode() == build.source_digest()
    assert len(build.sources()) >= 8 and any(s.endswith("sfdd.h") for s in build.sources())


def test_config_struct_layout_matches_header(tmp_path):
    # the binding's ctypes sf_config against the C compiler's layout of the header
    fields = [f[0] for f in api.sf_config._fields_]
    cname = {"lambda_": "lambda"}
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%s %zu\\n", "{f}", offsetof(sf_config, {cname.get(f, f)}));\n' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sfdd.h"\nint main(void) {\n'
                   '    printf("size %zu\\n", sizeof(sf_config));\n' + body + "    return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    import ctypes
    assert int(out["size"]) == ctypes.sizeof(api.sf_config)
    for f in fields:
        assert int(out[f]) == getattr(api.sf_config, f).offset, f


def test_config_validation_host_only():
    # sf_memory_bytes validates the configuration without a device
    import ctypes
    _ensure_built()
    n = ctypes.c_int64()
    good = api.make_config(64, 64, 1, 2, 2, 4, deferred_status=1)
    assert api.lib().sf_memory_bytes(ctypes.byref(good), ctypes.byref(n)) == api.SF_OK and n.value > 0
    for bad in (api.make_config(64, 64, 1, 2, 2, 4, deferred_status=2),
                api.make_config(64, 64, 1, 2, 2, 4, pivot_tol=1.0),
                api.make_config(64, 64, 1, 2, 2, 4, factor_precision=3),
                api.make_config(64, 64, 1, 2, 2, 4, rho=-1.0)):
        assert api.lib().sf_memory_bytes(ctypes.byref(bad), ctypes.byref(n)) == api.SF_ERR_INVALID


def test_null_context_calls_are_invalid_host_only():
    # entry points given no context return SF_ERR_INVALID without touching a device
    _ensure_built()
    lib = api.lib()
    assert lib.sf_set_wait_limit(None, 10) == api.SF_ERR_INVALID
    assert lib.sf_sync(None) == api.SF_ERR_INVALID
    assert lib.sf_factor_subdomains(None) == api.SF_ERR_INVALID
