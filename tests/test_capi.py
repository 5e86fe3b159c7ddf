"""The C ABI without a GPU: the library loads, exports every entry point the
public headers declare, and validates arguments before touching a device."""
import ctypes
import glob
import os
import re

import pytest

import paper_2208_01243_amd as aim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(aim_\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(aim.LIB_PATH)
    names = declared_symbols()
    assert "aim_align_batch" in names and "aim_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_abi():
    assert set(declared_symbols()) <= set(aim.SIGNATURES)


def test_version_and_error_string():
    assert "gfx950" in aim.version()
    assert aim.lib().aim_last_error() is not None


def _call(alg=aim.SWG_AFFINE, pen=(0, 4, 6, 2), n=1, max_len=10, want=1, cap=10, ctx=None, nulls=False):
    L = aim.lib()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    b = aim.Batch(n, aim.ENC_2BIT, max_len, *( [None] * 6 if nulls else [dummy] * 6))
    r = aim.Results(dummy, dummy, dummy, dummy, cap, want)
    return L.aim_align_batch(ctx, ctypes.byref(b), alg, aim.Penalties(*pen), -1, ctypes.byref(r), None)


@pytest.mark.parametrize("pen,code", [((1, 4, 6, 2), -2), ((0, 0, 6, 2), -1), ((0, 4, -1, 2), -1),
                                      ((0, 4, 6, 0), -1), ((0, 70000, 6, 2), -1)])
def test_penalty_validation(pen, code):
    assert _call(pen=pen) == code
    assert aim.lib().aim_last_error()


def test_linear_nw_rejects_gap_open():
    assert _call(alg=aim.NW_LINEAR, pen=(0, 1, 1, 1)) == -1
    assert b"gap_open" in aim.lib().aim_last_error()


def test_argument_validation():
    assert _call(alg=7) == -1
    assert _call(n=-1) == -1
    assert _call(max_len=-1) == -1
    assert _call(max_len=(1 << 20) + 1) == -1
    assert _call(nulls=True) == -1
    assert _call(cap=-1) == -1
    # everything valid but no context
    assert _call() == -1 and b"ctx" in aim.lib().aim_last_error()
    L = aim.lib()
    assert L.aim_align_batch(None, None, 0, aim.Penalties(0, 1, 0, 1), -1, None, None) == -1
    assert L.aim_create(None, 0, None) == -1


def test_pack_validation():
    L = aim.lib()
    assert L.aim_pack_2bit(None, 1, aim.ENC_ASCII, None, None, None, None, 0, None, None, None) == -1
