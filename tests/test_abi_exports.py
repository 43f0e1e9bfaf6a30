"""The C ABI library loads without a GPU and exports every function that
include/idcur.h declares; host-only entry points behave as documented.

No compute call is made here (those need a GPU and live in the gpu-marked
parity tests). The library is built first when it is missing.
"""
from __future__ import annotations

import ctypes
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "idcur.h")
PKG = os.path.join(ROOT, "paper_1412_8447_amd")
LIB = os.path.join(PKG, "libidcur.so")


def _declared():
    text = open(HEADER).read()
    # drop comments, then take every identifier idcur_* directly followed by "("
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(idcur_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        spec = importlib.util.spec_from_file_location("idcur_build", os.path.join(PKG, "build.py"))
        b = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(b)
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("idcur_id_col", "idcur_id_row", "idcur_id_two_sided", "idcur_cur", "idcur_workspace_bytes",
                 "idcur_create", "idcur_destroy", "idcur_sync_status", "idcur_gaussian"):
        assert must in names, must


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, f"declared in idcur.h but not exported: {missing}"


def test_binding_covers_the_header():
    src = open(os.path.join(PKG, "__init__.py")).read()
    m = re.search(r"EXPORTED\s*=\s*\((.*?)\)", src, flags=re.S)
    assert m
    bound = set(re.findall(r'"(idcur_\w+)"', m.group(1)))
    assert bound == set(_declared())


class _Opts(ctypes.Structure):
    # layout of idcur_opts as declared in the header
    _fields_ = [("k", ctypes.c_int32), ("kmax", ctypes.c_int32), ("tol", ctypes.c_double),
                ("rank_tol", ctypes.c_double), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("omega", ctypes.c_void_p), ("prec", ctypes.c_int32),
                ("norms", ctypes.c_int32), ("sketch", ctypes.c_int32), ("srht_signs", ctypes.c_void_p),
                ("srht_rows", ctypes.c_void_p), ("u_correct", ctypes.c_int32), ("t_reg", ctypes.c_double),
                ("t_svd", ctypes.c_double)]


def _opts_members():
    """Member names of idcur_opts in declaration order, from the header."""
    text = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    end = re.search(r"\}\s*idcur_opts\s*;", text)
    assert end, "idcur_opts not found in the header"
    body = text[text.rindex("{", 0, end.start()) + 1:end.start()]
    return [m.group(1) for m in re.finditer(r"(\w+)\s*;", body)]


def test_opts_mirror_matches_the_header():
    # idcur_opts_default writes the whole struct: a stale mirror here would let
    # it write past the Python-side buffer
    assert [f[0] for f in _Opts._fields_] == _opts_members()


def test_opts_default(lib):
    o = _Opts()
    ctypes.memset(ctypes.byref(o), 0x5A, ctypes.sizeof(o))
    lib.idcur_opts_default(ctypes.byref(o))
    assert (o.k, o.kmax, o.tol, o.rank_tol, o.p, o.q, o.seed) == (0, 0, 0.0, 0.0, -1, 0, 0)
    assert not o.omega and o.prec == 0 and o.norms == 0
    assert o.sketch == 0 and not o.srht_signs and not o.srht_rows and o.u_correct == 0 and o.t_reg == 0.0
    assert o.t_svd == 0.0


def test_null_context_is_rejected(lib):
    # argument checks happen before any device work
    lib.idcur_id_col.restype = ctypes.c_int
    o = _Opts()
    lib.idcur_opts_default(ctypes.byref(o))
    o.k = 2
    rc = lib.idcur_id_col(None, 1, ctypes.c_int64(8), ctypes.c_int64(8), None, ctypes.c_int64(8), ctypes.byref(o),
                          None, ctypes.c_size_t(0), None, None, None, ctypes.c_int64(0))
    assert rc == -1   # IDCUR_EINVAL
