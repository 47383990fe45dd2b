"""The C-ABI library loads and exports every entry point include/polrad.h
declares; the binding has no CPU fallback.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "polrad.h")).read()
    return sorted(set(re.findall(r"^\s*(?:kp_status|void|const char \*)\s*(kp_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("kp_create", "kp_destroy", "kp_set_grid", "kp_set_grid_device", "kp_set_dust",
                 "kp_set_source", "kp_set_views", "kp_run", "kp_transport", "kp_image",
                 "kp_image_source", "kp_get_images", "kp_get_images_device", "kp_get_stats",
                 "kp_get_trace", "kp_get_tally", "kp_last_error"):
        assert must in names


CITATION = re.compile(r"Sec\. \d|Appendix|App\. A|eq\. [a-z]|not in the paper|callers that cannot")


def declaration_comments(path):
    """(name, comment) for every entry point of a header: the comment block
    between the previous declaration and this one; a declaration with no
    comment of its own shares the one of the declaration before it."""
    txt = open(path).read()
    body = txt[txt.index('extern "C" {'):]
    out, prev_end, prev_comment = [], 0, ""
    for m in re.finditer(r"^\s*(?:kp_status|void|const char \*)\s*(kp_\w+)\s*\([^;]*;", body, re.M):
        gap = body[prev_end:m.start()]
        # comments that open a line (not the trailing comments of struct fields)
        comments = re.findall(r"^[ \t]*(/\*.*?\*/)", gap, re.M | re.S)
        if comments:
            prev_comment = re.sub(r"\s*\n\s*\*?\s*", " ", comments[-1])
        out.append((m.group(1), prev_comment))
        prev_end = m.end()
    return out


@pytest.mark.parametrize("header", ["polrad.h", "polrad_denoiser.h"])
def test_every_declaration_cites_its_passage(header):
    """Each entry point's comment names the passage of the paper that defines
    the operation (section, equation or appendix), or says that the learned
    denoiser is not in the paper."""
    decl = declaration_comments(os.path.join(ROOT, "include", header))
    assert len(decl) >= 10
    missing = [n for n, c in decl if not CITATION.search(c)]
    assert not missing, missing


def test_library_exports_every_declared_symbol():
    from paper_2512_01283_amd import polrad as P
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(P.header_symbols()) == declared()


def test_struct_layouts_match_header():
    from paper_2512_01283_amd import polrad as P
    # sizes implied by the C declarations (x86-64 SysV alignment)
    assert ctypes.sizeof(P.kp_grid) == 3 * 4 + 4 + 4 * 8 + 4 + 4
    assert ctypes.sizeof(P.kp_dust) == 7 * 8
    assert ctypes.sizeof(P.kp_source) == 8 + 7 * 8
    assert ctypes.sizeof(P.kp_view) == 2 * 8 + 2 * 4 + 8
    assert ctypes.sizeof(P.kp_opts) == 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 4 + 4
    assert P.TRACE_DTYPE.itemsize == 8 + 4 + 4 + 8 + 8 + 24 + 32 + 8 + 8
    # kp_stats: 8 int64 counters, 7 energies and 2 times (double), packets, tally_flushes
    assert ctypes.sizeof(P.kp_stats) == 8 * 8 + 9 * 8 + 2 * 8


def test_stats_fields_follow_the_header_order():
    import re
    from paper_2512_01283_amd import polrad as P
    txt = open(P.HEADER).read()
    body = txt[txt.index("typedef struct {", txt.index("Counters of the last")):txt.index("} kp_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"([a-z_0-9]+)\s*[,;]", body)
    assert names == [k for k, _ in P.kp_stats._fields_]


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_calibration_library_exports_its_entry_point():
    from paper_2512_01283_amd import build as B
    if not os.path.exists(B.CALIB_LIB):
        pytest.skip("libkpcalib.so not built")
    lib = ctypes.CDLL(B.CALIB_LIB)
    assert hasattr(lib, "kpcal_atomic_lines")


def test_no_device_is_reported_cleanly():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    from paper_2512_01283_amd import polrad as P
    h = ctypes.c_void_p()
    assert P._lib.kp_create(0, ctypes.byref(h)) == P.KP_ERR_DEVICE
    assert P._lib.kp_set_grid(None, None, None, None) == P.KP_ERR_ARG
    assert P._lib.kp_run(None, None, None, None) == P.KP_ERR_ARG


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    src = os.path.join(ROOT, "paper_2512_01283_amd", "polrad.py")
    dst = tmp_path / "polrad.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("polrad_copy", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def declared_denoiser():
    txt = open(os.path.join(ROOT, "include", "polrad_denoiser.h")).read()
    return sorted(set(re.findall(r"^\s*(?:kp_status|void|const char \*)\s*(kp_\w+)\s*\(", txt, re.M)))


def test_denoiser_header_symbols_exported_and_bound():
    from paper_2512_01283_amd import denoiser as DN
    names = declared_denoiser()
    for must in ("kp_dn_create", "kp_dn_destroy", "kp_dn_infer", "kp_dn_backward", "kp_dn_adam_step",
                 "kp_dn_train_step", "kp_dn_set_params", "kp_dn_get_params", "kp_dn_get_grads",
                 "kp_dn_get_adam", "kp_dn_set_adam", "kp_dn_num_params", "kp_dn_last_error",
                 "kp_dn_get_timing"):
        assert must in names
    lib = ctypes.CDLL(DN.P.LIB_PATH)
    assert not [n for n in names if not hasattr(lib, n)]
    assert DN.header_symbols() == names
    assert sorted(DN._SIGS) == names
    assert ctypes.sizeof(DN.kp_dn_timing) == 6 * 8


def test_denoiser_without_device_and_bad_arguments():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    from paper_2512_01283_amd import denoiser as DN
    import numpy as np
    h = ctypes.c_void_p()
    good = np.array([48, 96, 192], np.int32)
    bad = np.array([40, 96, 192], np.int32)
    assert DN._lib.kp_dn_create(0, good.ctypes.data, 3, ctypes.byref(h)) == DN.P.KP_ERR_DEVICE
    assert DN._lib.kp_dn_create(0, bad.ctypes.data, 3, ctypes.byref(h)) == DN.P.KP_ERR_ARG
    assert DN._lib.kp_dn_create(0, good.ctypes.data, 1, ctypes.byref(h)) == DN.P.KP_ERR_ARG
    assert DN._lib.kp_dn_create(0, good.ctypes.data, 7, ctypes.byref(h)) == DN.P.KP_ERR_ARG
    assert DN._lib.kp_dn_infer(None, None, None, 1, 16, 16, None) == DN.P.KP_ERR_ARG
    assert DN._lib.kp_dn_num_params(None, None) == DN.P.KP_ERR_ARG


def test_packets_to_fixed_error_interpolation():
    """The evaluation's N_den: log-log interpolation between the counts that
    bracket eps, the smallest count if eps is already met there, NaN if it
    is never met."""
    import math

    from paper_2512_01283_amd.dn_train import _packets_to_eps
    counts = (1e5, 1e6, 1e7)
    errs = {1e5: 0.1, 1e6: 0.1 / math.sqrt(10), 1e7: 0.01}  # E = a N^-1/2
    n, b = _packets_to_eps(counts, errs, 0.02)
    assert b == "=" and abs(n - 2.5e6) < 1e-6 * 2.5e6  # (0.1 / 0.02)^2 * 1e5
    assert _packets_to_eps(counts, errs, 0.2) == (1e5, "<=")
    n, b = _packets_to_eps(counts, errs, 0.005)
    assert b == "not reached" and n != n
