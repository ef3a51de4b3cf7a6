"""Robustness of the library's front end (no GPU): random token soups as
statements, map expressions, reduce expressions and neutral elements come
back as a status (parse error, unsupported, hipRTC's rejection or success),
never as a crash, and every failure leaves a message."""

import ctypes
import random

import paper_1304_5553_amd as hm

EW_TOKENS = ["x[i]", "y[i]", "z[i]", "i", "n", "a", "+", "-", "*", "/", "%", "(", ")", "[", "]", "?",
             ":", "=", "==", "<", "&&", "||", "!", "~", "1", "2.5f", "0x1f", "sqrtf(", "max(", ",", ";",
             "x[i+1]", "x[i-n]", "y[3]", "(float)", "z[i] =", "+=", "{", "}", "if", "else", "float t =",
             "t", "'", "\"", "\\", "x[", "i]", "@", "#", "x[i + a]", "x[i*2]", "x[-i]", "1e40f", "0u"]
RED_TOKENS = ["x[i]", "k[i]", "i", "n", "+", "-", "*", "/", "%", "(", ")", "?", ":", "==", "<", "&&",
              "!", "1", "2.5f", "sqrtf(", "max(", ",", "x[i+1]", "k[i-2]", "x[4]", "(float)", "x[", "i]"]
ALLOWED = {0, -1, -2, -3, -6}


def test_random_statements_return_a_status(tmp_path, monkeypatch):
    monkeypatch.setenv("HIPMR_CACHE_DIR", str(tmp_path))     # keep the user's cache clean
    lib = hm.hipmr.lib()
    rng = random.Random(1)
    seen = set()
    for _ in range(150):
        expr = " ".join(rng.choice(EW_TOKENS) for _ in range(rng.randint(0, 10)))
        h = ctypes.c_void_p()
        st = lib.hipmr_compile(expr.encode(), b"float *z, const float *x, const float *y, float a",
                               ctypes.byref(h))
        assert st in ALLOWED, (expr, st)
        if st == 0:
            lib.hipmr_release(h)
        else:
            assert lib.hipmr_last_error(), expr
        seen.add(st)
    assert -2 in seen


def test_random_reductions_return_a_status(tmp_path, monkeypatch):
    monkeypatch.setenv("HIPMR_CACHE_DIR", str(tmp_path))
    lib = hm.hipmr.lib()
    rng = random.Random(2)
    for _ in range(80):
        expr = " ".join(rng.choice(RED_TOKENS) for _ in range(rng.randint(0, 6)))
        rt = rng.choice([b"float", b"long", b"double", b"unsigned", b"char", b"complex64"])
        h = ctypes.c_void_p()
        st = lib.hipmr_compile(expr.encode(), rt + b": const float *x, const int *k", ctypes.byref(h))
        if st == 0:
            st = lib.hipmr_prepare_reduce(h, rng.choice([b"a+b", b"max(a,b)", b"a*b", b"b+", b""]),
                                          rng.choice([b"0", b"-INFINITY", b"", b"x[i]", b"0)"]))
            lib.hipmr_release(h)
        assert st in ALLOWED, (expr, st)
