"""Argument checks of the C ABI on the CPU (no GPU): the library's checker
(paper_1412_8447_amd/csrc/args.cpp, which every entry point runs before it sizes
the workspace or enqueues work) is built alone with the address and
undefined-behaviour sanitizers and driven through every documented error code
of include/idcur.h: sizes, leading dimensions, rank and tolerance mode, sketch
width, precision and dtype, option enums, the structured sketch's requirements,
the outputs each operation writes, and the batched ID's limits.

The GPU test tests/test_gpu_abi_errors.py checks the same codes through the
shared library's entry points.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_8447_amd", "csrc")

OK, EINVAL, EDTYPE = 0, -1, -2
F64, F32 = 0, 1
BIG = "m=10000 n=10000 lda=10000"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("args") / "host_args_driver")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "args.cpp"), os.path.join(ROOT, "tests", "host_args_driver.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def run_cases(driver, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    outs = r.stdout.strip().split("\n")
    assert len(outs) == len(lines)
    res = []
    for o in outs:
        code, msg = o.split(" ", 1)
        res.append((int(code), msg))
    return res


# (input line, expected status, substring of the message)
ID_CASES = [
    ("id", OK, "-"),
    ("id opts=0", EINVAL, "opts is NULL"),
    ("id dtype=7", EDTYPE, "dtype"),
    ("id prec=5", EINVAL, "precision"),
    ("id prec=1", EDTYPE, "FP32"),
    ("id prec=2", EDTYPE, "FP32"),
    (f"id dtype={F32} prec=1 p=4", OK, "-"),
    ("id op=9", EINVAL, "op"),
    ("id op=-1", EINVAL, "op"),
    ("id m=0", EINVAL, "positive"),
    ("id n=0", EINVAL, "positive"),
    ("id m=2000000000", EINVAL, "2^30"),
    ("id n=2000000000 lda=2000000000", EINVAL, "2^30"),
    ("id lda=47", EINVAL, "lda"),
    ("id k=-1", EINVAL, "k must be >= 0"),
    ("id k=48", EINVAL, "min(m, n)"),
    ("id k=47", OK, "-"),
    ("id k=0 tol=0 kmax=10", EINVAL, "tol > 0"),
    ("id k=0 tol=nan kmax=10", EINVAL, "tol > 0"),
    ("id k=0 tol=inf kmax=10", EINVAL, "tol > 0"),
    ("id k=0 tol=1e-3 kmax=0", EINVAL, "kmax"),
    ("id k=0 tol=1e-3 kmax=48", EINVAL, "kmax"),
    ("id k=0 tol=1e-3 kmax=47", OK, "-"),
    ("id q=-1", EINVAL, "q must be"),
    (f"id {BIG} k=5000", EINVAL, "4096"),
    (f"id {BIG} k=5 p=5000", EINVAL, "4096"),
    (f"id {BIG} k=4000 p=96", OK, "-"),
    ("id op=4 p=-1", EINVAL, "a sketch needs"),
    ("id op=4 p=100", EINVAL, "a sketch needs"),
    ("id op=4 p=4", OK, "-"),
    ("id op=5 p=43", EINVAL, "a sketch needs"),   # row sketch: k + p below n = 48
    ("id op=5 p=42", OK, "-"),
    ("id rank_tol=-1", EINVAL, "rank_tol"),
    ("id rank_tol=inf", EINVAL, "rank_tol"),
    ("id norms=7", EINVAL, "norms"),
    ("id norms=1", OK, "-"),
    ("id sketch=9", EINVAL, "sketch kind"),
    ("id u_correct=2", EINVAL, "u_correct"),
    ("id t_reg=1.5", EINVAL, "t_reg"),
    ("id t_reg=1.0", EINVAL, "t_reg"),
    ("id t_reg=-0.1", EINVAL, "t_reg"),
    ("id t_reg=nan", EINVAL, "t_reg"),
    ("id t_reg=0.001", OK, "-"),
    ("id t_svd=1.5", EINVAL, "t_svd"),
    ("id t_svd=-1e-3", EINVAL, "t_svd"),
    ("id t_svd=nan", EINVAL, "t_svd"),
    ("id t_svd=1e-6", EINVAL, "switched off"),
    ("id t_reg=1e-3 t_svd=1e-6", EINVAL, "exclude each other"),
    ("id sketch=1 p=4 q=1 srht_rows=1 srht_signs=1", EINVAL, "power steps"),
    (f"id dtype={F32} sketch=1 p=4 prec=1 srht_rows=1 srht_signs=1", EDTYPE, "native precision"),
    ("id sketch=1 p=4 omega=1 srht_rows=1 srht_signs=1", EINVAL, "exclude"),
    ("id sketch=1 p=4", EINVAL, "required"),
    ("id sketch=1 p=4 srht_rows=1", EINVAL, "required"),
    ("id sketch=1 p=4 srht_rows=1 srht_signs=1", OK, "-"),
    ("id sketch=1 p=600 m=2000 n=2000 lda=2000 srht_rows=1 srht_signs=1", EINVAL, "512"),
    ("id sketch=1 p=-1", OK, "-"),   # no sketch taken: the kind is not used
]

OUTS_CASES = [
    ("outs", OK, "-"),
    ("outs A=0", EINVAL, "A is NULL"),
    ("outs op=4 p=4 Yt=0", EINVAL, "Yt"),
    ("outs op=4 p=4 ldy=8", EINVAL, "ldy"),
    ("outs op=4 p=4 ldy=9", OK, "-"),
    ("outs k_out=0", EINVAL, "k_out"),
    ("outs op=1 I=0", EINVAL, "I and Tr"),
    ("outs op=1 Tr=0", EINVAL, "I and Tr"),
    ("outs op=1 ldtr=58", EINVAL, "ldtr"),
    ("outs op=1 ldtr=59", OK, "-"),
    ("outs op=1 J=0 T=0", OK, "-"),   # the row ID writes I and Tr only
    ("outs J=0", EINVAL, "J is required"),
    ("outs T=0", EINVAL, "T is required"),
    ("outs ldt=42", EINVAL, "ldt"),
    ("outs ldt=43", OK, "-"),
    ("outs k=0 tol=1e-3 kmax=10 ldt=47", EINVAL, "ldt"),
    ("outs k=0 tol=1e-3 kmax=10 ldt=48", OK, "-"),
    ("outs op=2 Tr=0", EINVAL, "I and Tr"),
    ("outs op=2 ldtr=58", EINVAL, "ldtr"),
    ("outs op=2 U=0 C=0 R=0", OK, "-"),
    ("outs op=3 U=0", EINVAL, "I and U"),
    ("outs op=3 I=0", EINVAL, "I and U"),
    ("outs op=3 ldu=4", EINVAL, "ldu"),
    ("outs op=3 ldc=4", EINVAL, "ldc"),
    ("outs op=3 C=0 ldc=4", OK, "-"),
    ("outs op=3 ldr=47", EINVAL, "ldr"),
    ("outs op=3 R=0 ldr=47", OK, "-"),
    ("outs op=3 T=0 Tr=0", OK, "-"),   # the CUR keeps T internal
]

BATCHED_CASES = [
    ("batched", OK, "-"),
    ("batched opts=0", EINVAL, "opts is NULL"),
    (f"batched dtype={F64}", EDTYPE, "FP32"),
    ("batched prec=1", EDTYPE, "FP32"),
    ("batched nblk=-1", EINVAL, "nblk"),
    ("batched nblk=2000000", EINVAL, "nblk"),
    ("batched nblk=0", OK, "-"),
    ("batched mmax=0", EINVAL, "mmax"),
    ("batched mmax=20000000", EINVAL, "mmax"),
    ("batched nmax=0", EINVAL, "nmax"),
    ("batched nmax=513", EINVAL, "nmax"),
    ("batched nmax=512", OK, "-"),
    ("batched p=0", EINVAL, "oversampling"),
    ("batched q=1", EINVAL, "power steps"),
    ("batched k=-1", EINVAL, "k must be"),
    ("batched k=0 tol=0 kmax=5", EINVAL, "tol > 0"),
    ("batched k=0 tol=1e-6 kmax=0", EINVAL, "kmax"),
    ("batched k=0 tol=1e-6 kmax=8", OK, "-"),
    ("batched k=61 p=4", EINVAL, "64"),
    ("batched k=60 p=4", OK, "-"),
    ("batched rank_tol=-1", EINVAL, "rank_tol"),
    ("batched t_reg=0.1", EINVAL, "t_reg"),
    ("batched t_svd=0.1", EINVAL, "t_svd"),
]


@pytest.mark.parametrize("cases", [ID_CASES, OUTS_CASES, BATCHED_CASES], ids=["id", "outs", "batched"])
def test_error_codes(driver, cases):
    got = run_cases(driver, [c[0] for c in cases])
    for (line, code, sub), (gc, gm) in zip(cases, got):
        assert gc == code, (line, gc, gm)
        if code == OK:
            assert gm == "-", line
        else:
            assert sub in gm, (line, gm)


def test_every_error_line_is_reached(driver):
    """Each distinct message of the checker appears among the cases above, so
    no branch is left untested."""
    src = open(os.path.join(CSRC, "args.cpp")).read()
    msgs = set(re.findall(r'(?:inval|dtype_err)\("([^"]+)"\)', src))
    lines = [c[0] for c in ID_CASES + OUTS_CASES + BATCHED_CASES]
    got = {m for _, m in run_cases(driver, lines)}
    missing = sorted(m for m in msgs if m not in got)
    assert not missing, missing

