"""CPU tests of the C ABI library: it loads, exports every symbol the
header declares, and its host logic (signature parser, expression
classifier, code generation, hipRTC compile cache, SHA-256, error codes)
behaves.  No kernel is launched here."""

import ctypes
import hashlib
import os
import re

import pytest

import paper_1304_5553_amd as hm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hipmr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hipmr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(hm.hipmr.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(declared_functions()) <= set(hm.hipmr._SIGS)


@pytest.mark.parametrize("data", [b"", b"abc", b"a" * 55, b"a" * 56, b"a" * 64, b"x" * 1000,
                                  bytes(range(256)) * 3])
def test_sha256_matches_hashlib(data):
    assert hm.sha256_hex(data) == hashlib.sha256(data).hexdigest()


def test_classifier_read_write_sets():
    k = hm.compile("z[i] = 2.5f*x[i] - 0.5f*y[i]", "float *z, const float *x, const float *y")
    assert k.vectorizable and k.vec == 4
    assert [(a.read, a.written) for a in k.args] == [(0, 1), (1, 0), (1, 0)]
    k = hm.compile("a[i] *= 2", "float *a")
    assert [(a.read, a.written) for a in k.args] == [(1, 1)]
    k = hm.compile("if (x[i] > 0) z[i] = 1; else z[i] = 2", "float *z, const float *x")
    assert k.vectorizable
    src = k.source(0)
    assert "hipmr_load<HIPMR_NTL>(hipmr_p_z" in src          # conditional write: z is loaded first
    k = hm.compile("z[i] = x[i * 2]", "float *z, const float *x")
    assert not k.vectorizable
    k = hm.compile("q[i] = x[i]", "fp8_e4m3 *q, const bfloat16 *x")
    assert k.vec == 16                                 # 16 bytes of the narrowest array


def test_fixed_element_reads_stay_on_the_vector_path():
    # a device-resident scalar read as a[0] is the same element for every i:
    # read directly, never moved in chunks, and it does not narrow VEC
    k = hm.compile("x[i] += a[0] * p[i]", "float *x, const float *p, const double *a")
    assert k.vectorizable and k.vec == 4
    assert [(a.read, a.written) for a in k.args] == [(1, 1), (1, 0), (1, 0)]
    src = k.source(0)
    assert "hipmr_p_p[hipmr_u].v[hipmr_j]" in src and "a [ 0 ]" in src
    assert "hipmr_p_a" not in src
    r = hm.compile("s[1] * x[i]", "float: const float *x, const fp8_e4m3 *s")
    assert r.vectorizable and r.vec == 4               # fp8 s is not chunked
    # writing the array elsewhere keeps the one-element path
    k = hm.compile("z[i] = z[0] + 1", "float *z")
    assert not k.vectorizable
    k = hm.compile("z[i] = x[n - 1]", "float *z, const float *x")
    assert not k.vectorizable


def test_shifted_reads_classification():
    # name[i + E] / name[i - E] with E uniform (literals, scalar arguments, n)
    # reads an array at the same distance for every i: elementwise statements
    # keep the vector kernel, with one unaligned chunk load per distinct read
    sig = "float *q, const float *p, int nx"
    stmt = ("int c = i % nx; q[i] = 4.0f*p[i] - (c != 0 ? p[i-1] : 0.0f) - (c != nx - 1 ? p[i+1] : 0.0f)"
            " - (i >= nx ? p[i-nx] : 0.0f) - (i + nx < n ? p[i+nx] : 0.0f)")
    k = hm.compile(stmt, sig)
    assert k.vectorizable and k.vec == 4
    src = k.source(0)
    for r, off in enumerate(("(0 - 1)", "(0 + 1)", "(0 - nx)", "(0 + nx)")):
        assert f"hipmr_s{r} = (long long){off}" in src
        assert f"hipmr_loadu(hipmr_q{r}[hipmr_u], p + hipmr_off + hipmr_s{r})" in src
    assert "hipmr_q4" not in src                       # four distinct distances
    assert "hipmr_load<HIPMR_NTL>(hipmr_p_p" in src    # p[i] itself: an aligned chunk
    # a repeated read shares its load; bfloat16 narrows VEC to 8
    k = hm.compile("o[i] = x[i + 2*k] + x[i + 2*k] * x[i - (k)]", "float *o, const bfloat16 *x, long k")
    assert k.vectorizable and k.vec == 8
    assert "hipmr_q1" in k.source(0) and "hipmr_q2" not in k.source(0)
    # no shifted reads: the source of a plain kernel does not change
    plain = hm.compile("z[i] = 2.5f*x[i] - 0.5f*y[i]", "float *z, const float *x, const float *y")
    assert "hipmr_loadu" not in plain.source(0)
    # cases that keep the one-element kernel
    for stmt, sig in (("x[i] = x[i + 1]", "float *x"),                        # shifted array written
                      ("int c = 1; z[i] = x[i + c]", "float *z, const float *x"),   # local in E
                      ("z[i] = x[i + nx << 1]", "float *z, const float *x, int nx"),  # (i + nx) << 1
                      ("z[i] = x[i + y[0]]", "float *z, const float *x, const int *y"),  # array in E
                      ("z[i] = x[i + i]", "float *z, const float *x")):
        assert not hm.compile(stmt, sig).vectorizable, stmt
    assert hm.compile("z[i] = x[i + (nx << 1)]", "float *z, const float *x, int nx").vectorizable
    # maps: the plain reduce loads shifted reads as chunks too
    r = hm.compile("(i + 1 < n ? x[i + 1] : 0.0f) - x[i]", "float: const float *x")
    assert r.vectorizable
    assert ("hipmr_loadu(hipmr_q0[hipmr_u], x + hipmr_clampv(hipmr_off, hipmr_s0, hipmr_n - HIPMR_V))"
            in r.source(2, "a+b", "0"))


def test_argument_access_flags_and_length_check():
    import torch
    A = hm.hipmr
    k = hm.compile("x[i] += (float)a[0] * p[i] + (i >= 1 ? p[i - 1] : 0.0f) + q[n - 1 - i]",
                   "float *x, const float *p, const double *a, const float *q")
    assert [a.access for a in k.args] == [A.ACCESS_INDEX, A.ACCESS_INDEX | A.ACCESS_SHIFTED,
                                         A.ACCESS_FIXED, A.ACCESS_OTHER]
    # arrays indexed by i (or i +/- E) need n elements; fixed-element arrays do not
    x, p, a, q = torch.zeros(10), torch.zeros(10), torch.zeros(1, dtype=torch.float64), torch.zeros(3)
    k.check_lengths(10, [x, p, a, q])
    with pytest.raises(hm.InvalidError, match="'p' has 9 elements"):
        k.check_lengths(10, [x, p[:9], a, q])
    s = hm.compile("(i + 2 < n ? y[i + 2] : 0.0f)", "float: const float *y")
    assert s.args[0].access == A.ACCESS_SHIFTED
    with pytest.raises(hm.InvalidError):
        s.check_lengths(11, [torch.zeros(10)])
    assert hm.compile("x[i]", "float: const float *x, float c").args[1].access == 0   # a scalar


def test_marshal_holds_each_value_in_its_c_type():
    # args[k] points at the bytes of argument k as its C type (wrapping
    # integers, float overflow to inf, low-precision scalars rounded once)
    import torch
    B = hm.hipmr
    sig = ("float *z, float a, double b, char c, unsigned char d, short e, unsigned short f, int g, "
           "unsigned h, long l, bfloat16 m, half o, fp8_e4m3 q, complex64 r")
    k = hm.compile("z[i] = a", sig)
    vals = [torch.zeros(4), 1.0e300, -2.5, -3, 300, -40000, 70000, 2 ** 31 + 5, -1, -(2 ** 40), 1.5,
            131008.0, 500.0, 0.25 - 1.5j]
    store, ptrs = k.marshal(vals)
    want = [ctypes.c_void_p(vals[0].data_ptr()), ctypes.c_float(vals[1]), ctypes.c_double(vals[2]),
            ctypes.c_int8(vals[3]), ctypes.c_uint8(vals[4]), ctypes.c_int16(vals[5]),
            ctypes.c_uint16(vals[6]), ctypes.c_int32(vals[7]), ctypes.c_uint32(vals[8]),
            ctypes.c_int64(vals[9]), ctypes.c_uint16(0x3FC0), ctypes.c_uint16(0x7C00),
            ctypes.c_uint8(0x7E), (ctypes.c_float * 2)(0.25, -1.5)]
    for i, w in enumerate(want):
        assert ctypes.string_at(ptrs[i], ctypes.sizeof(w)) == bytes(w), i
    with pytest.raises(hm.InvalidError):
        k.marshal(vals[:-1])


def test_marshal_reuses_one_buffer_per_thread():
    # the library copies argument values during the call, so a handle keeps
    # one pair of buffers per thread; the next call rewrites every slot
    import threading

    import torch
    k = hm.compile("z[i] = a * x[i] + b", "float *z, float a, const float *x, long b")
    z, x = torch.zeros(4), torch.ones(4)
    s1, p1 = k.marshal([z, 2.5, x, -7])
    addr = ctypes.addressof(s1)
    s2, p2 = k.marshal([x, -0.5, z, 2 ** 40])
    assert ctypes.addressof(s2) == addr and p2[0] == addr
    want = [ctypes.c_void_p(x.data_ptr()), ctypes.c_float(-0.5), ctypes.c_void_p(z.data_ptr()),
            ctypes.c_int64(2 ** 40)]
    for i, w in enumerate(want):
        assert ctypes.string_at(p2[i], ctypes.sizeof(w)) == bytes(w), i
    other = []
    t = threading.Thread(target=lambda: other.append(ctypes.addressof(k.marshal([z, 1.0, x, 1])[0])))
    t.start()
    t.join()
    assert other and other[0] != addr


def test_generated_source_shape():
    k = hm.compile("z[i] = 2.5f*x[i] - 0.5f*y[i]", "float *z, const float *x, const float *y",
                   name="lin")
    src = k.source(0)
    assert 'extern "C" __global__' in src and "__launch_bounds__(256)" in src
    assert re.search(r"lin_ew_[0-9a-f]{8}\(", src)
    assert "hipmr_p_x[hipmr_u].v[hipmr_j]" in src
    assert "hipmr_load<HIPMR_NTL>(hipmr_p_z" not in src       # write-only: never loaded
    r = hm.compile("x[i]", "float: const float *x", name="mx")
    s1 = r.source(2, "max(a,b)", "-INFINITY")
    assert "__builtin_elementwise_maximum(a, b)" in s1 and "hipmr_block_reduce" in s1
    s2 = r.source(4, "a+b", "0")
    assert "hipmr_partial[k]" in s2
    with pytest.raises(hm.MismatchError):
        r.source(0)


@pytest.mark.parametrize("expr,dtypes,exc", [
    ("z[i] = x[i]", "float *z, const quux *x", hm.ParseError),
    ("z[i] = x[i]", "float *z, float *z", hm.ParseError),
    ("z[i] = x[i]", "float *i, const float *x", hm.ParseError),
    ("z[i] = x[i] +* 2", "float *z, const float *x", hm.CompileError),
    ("return; z[i] = 1", "float *z", hm.UnsupportedError),
    ("z[i] = (x[i]", "float *z, const float *x", hm.ParseError),
    ("x[i] = 1", "float: float *x", hm.UnsupportedError),
    ("x[i] = 1", "const float *x", hm.ParseError),
    ("x[i]", "bfloat16: const float *x", hm.UnsupportedError),
    ("a = 2; z[i] = a", "float *z, float a", hm.UnsupportedError),
])
def test_errors_map_to_exceptions(expr, dtypes, exc):
    with pytest.raises(exc) as e:
        hm.compile(expr, dtypes)
    assert str(e.value)


def test_compile_error_carries_the_hiprtc_log():
    with pytest.raises(hm.CompileError) as e:
        hm.compile("z[i] = undefined_thing(x[i])", "float *z, const float *x")
    assert "undefined_thing" in str(e.value)


def test_compile_cache_memory_and_disk(tmp_path, monkeypatch):
    # a source the process has not seen: first a compile, then memory hits
    tag = os.urandom(4).hex()
    expr = f"z[i] = x[i] * 3.0f + {int(tag, 16) % 1000}"
    s0 = hm.cache_stats()
    hm.compile(expr, "float *z, const float *x")
    s1 = hm.cache_stats()
    assert s1["compiles"] + s1["disk_hits"] == s0["compiles"] + s0["disk_hits"] + 1
    hm.compile(expr, "float *z, const float *x")
    s2 = hm.cache_stats()
    assert s2["memory_hits"] == s1["memory_hits"] + 1 and s2["compiles"] == s1["compiles"]
    # after dropping the memory cache the same source loads from disk
    hm.cache_drop_memory()
    hm.compile(expr, "float *z, const float *x")
    s3 = hm.cache_stats()
    assert s3["disk_hits"] == s2["disk_hits"] + 1 and s3["compiles"] == s2["compiles"]


def test_compile_returns_the_cached_handle_and_release_balances():
    """compile() of the same (name, dtypes, expression) while a reference is
    held returns the same handle and touches neither the front end nor the
    code-object cache; once every reference is released the next compile()
    builds a new handle (its code object found in the memory cache)."""
    import gc
    tag = os.urandom(4).hex()
    expr, sig = f"z[i] = x[i] + {int(tag, 16) % 9973}", "float *z, const float *x"
    k1 = hm.compile(expr, sig, name="cached")
    s0 = hm.cache_stats()
    k2 = hm.compile(expr, sig, name="cached")
    k3 = hm.compile(expr, sig, name="cached")
    assert k1.handle.value == k2.handle.value == k3.handle.value
    assert hm.cache_stats() == s0                          # a handle hit: no cache lookup at all
    other = hm.compile(expr, sig, name="cached_other")     # another name is another handle
    assert other.handle.value != k1.handle.value
    del k2, k3
    gc.collect()
    k4 = hm.compile(expr, sig, name="cached")              # k1 still holds a reference
    assert k4.handle.value == k1.handle.value and hm.cache_stats()["memory_hits"] == s0["memory_hits"]
    del k1, k4
    gc.collect()
    s1 = hm.cache_stats()
    k5 = hm.compile(expr, sig, name="cached")              # all released: built again
    s2 = hm.cache_stats()
    assert s2["memory_hits"] == s1["memory_hits"] + 1 and s2["compiles"] == s1["compiles"]
    # after the memory caches are dropped, compile() builds a new handle (from disk)
    hm.cache_drop_memory()
    k6 = hm.compile(expr, sig, name="cached")
    assert k6.handle.value != k5.handle.value
    assert hm.cache_stats()["disk_hits"] == s2["disk_hits"] + 1
    del k5, k6, other


def test_corrupt_disk_entry_is_rebuilt():
    cache = os.environ.get("HIPMR_CACHE_DIR") or os.path.join(
        os.environ.get("XDG_CACHE_HOME") or os.path.expanduser("~/.cache"), "hipmr")
    tag = os.urandom(4).hex()
    expr = f"z[i] = x[i] - {int(tag, 16) % 100000}"
    hm.compile(expr, "float *z, const float *x")
    newest = max((os.path.join(cache, f) for f in os.listdir(cache) if f.endswith(".hsaco")),
                 key=os.path.getmtime)
    with open(newest, "r+b") as f:
        f.seek(200)
        f.write(b"\x00garbage\x00")
    hm.cache_drop_memory()
    s0 = hm.cache_stats()
    hm.compile(expr, "float *z, const float *x")
    s1 = hm.cache_stats()
    assert s1["disk_rejects"] == s0["disk_rejects"] + 1
    assert s1["compiles"] == s0["compiles"] + 1


def test_prepare_reduce_builds_without_a_gpu():
    k = hm.compile("k[i] % 7 == 3", "long: const int *k")
    hm.prepare_reduce(k, "a+b", "0")
    assert hm.reduce_workspace_bytes(k, 1 << 28) >= 8 * 2048


def test_selftest_compiles_every_template():
    assert hm.selftest_compile() >= 30


def test_missing_library_fails_loudly(monkeypatch):
    # the product path has no CPU or torch fallback: without the built
    # library every call raises
    monkeypatch.setattr(hm.hipmr, "LIB_PATH", "/nonexistent/libhipmr.so")
    monkeypatch.setattr(hm.hipmr, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        hm.compile("z[i] = x[i]", "float *z, const float *x")


def test_product_code_never_uses_the_oracle():
    # the oracle is test infrastructure: the package (Python and native
    # sources) neither imports nor names it, and shares none of its files
    import pathlib
    pkg = pathlib.Path(hm.__file__).resolve().parent
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.cpp")) + list(pkg.rglob("*.h")):
        text = f.read_text()
        assert "import oracle" not in text and "from oracle" not in text, f
        assert "oracle/" not in text, f


def test_server_config_validation_without_a_gpu():
    # the serving entry points check their arguments before any HIP call:
    # bad configurations, a missing or short workspace and NULL servers
    B = hm.hipmr
    L = B.lib()
    base = B.ServerConfig()
    need = L.hipmr_server_workspace_bytes(ctypes.byref(base))
    two = B.ServerConfig(nstreams=2)
    assert need > 0 and L.hipmr_server_workspace_bytes(ctypes.byref(two)) * 2 == need
    buf = ctypes.create_string_buffer(need)
    out = ctypes.c_void_p()
    for bad in (dict(nstreams=17), dict(nstreams=-1), dict(max_batch_jobs=4097),
                dict(max_batch_tiles=-1), dict(batch_backlog=-1),
                dict(max_batch_bytes=1 << 20, solo_bytes=2 << 20)):
        st = L.hipmr_server_create(ctypes.byref(B.ServerConfig(**bad)), buf, need, ctypes.byref(out))
        assert st == -1 and not out.value, bad
    assert L.hipmr_server_create(ctypes.byref(base), None, need, ctypes.byref(out)) == -8
    assert L.hipmr_server_create(ctypes.byref(base), buf, need - 1, ctypes.byref(out)) == -8
    assert L.hipmr_server_create(ctypes.byref(base), buf, need, None) == -1
    nd = ctypes.c_int32()
    t = ctypes.c_uint64()
    assert L.hipmr_server_poll(None, None, 0, ctypes.byref(nd)) == -1
    assert L.hipmr_server_submit(None, None, ctypes.byref(t)) == -1
    assert L.hipmr_server_wait_idle(None) == -1
    assert L.hipmr_server_run_schedule(None, None, 0, None) == -1
    L.hipmr_server_destroy(None)


def test_workspace_sizes_follow_their_documented_rules():
    # reduce: 64 KiB of block partials, 32 KiB of the norm's first-pass
    # partials and 256 bytes for its scale, whatever n; 0 for an
    # elementwise handle.  Segmented: grows with the number of segments and
    # elements (the tile table), never below the plain reduce's partials.
    red = hm.compile("k[i]", "long: const int *k")
    ew = hm.compile("z[i] = x[i]", "float *z, const float *x")
    sizes = {hm.reduce_workspace_bytes(red, n) for n in (0, 1, 1000, 1 << 20, 1 << 28, 1 << 40)}
    assert sizes == {65536 + 32768 + 256}
    assert hm.reduce_workspace_bytes(ew, 1 << 20) == 0
    seg = [hm.segmented_workspace_bytes(red, 4096, n) for n in (0, 1 << 20, 1 << 28)]
    assert seg == sorted(seg) and seg[0] > 0
    assert hm.segmented_workspace_bytes(red, 8192, 1 << 20) > hm.segmented_workspace_bytes(red, 4096, 1 << 20)


def test_binding_checks_outputs_and_offsets_before_the_library():
    """The C ABI takes bare pointers, so the binding checks what the library
    will write: the output tensor's dtype (the result type; none for an
    elementwise handle), contiguity and length, and the segmented offsets
    (int64, nseg + 1 values).  All of it is refused before any device work."""
    import torch
    r = hm.compile("x[i]", "float: const float *x", name="outchk")
    e = hm.compile("z[i] = x[i]", "float *z, const float *x", name="outchk_ew")
    x = torch.zeros(8)
    with pytest.raises(hm.MismatchError, match="elementwise handle"):
        hm.scan(e, "a+b", "0", 4, [x, x], torch.empty(4))
    with pytest.raises(hm.MismatchError, match="result type"):
        hm.scan(r, "a+b", "0", 4, [x], torch.empty(4, dtype=torch.float64))
    with pytest.raises(hm.InvalidError, match="4 are written"):
        hm.scan(r, "a+b", "0", 4, [x], torch.empty(3))
    with pytest.raises(hm.InvalidError, match="contiguous"):
        hm.scan(r, "a+b", "0", 4, [x], torch.empty(8)[::2])
    with pytest.raises(hm.MismatchError, match="result type"):
        hm.reduce(r, None, "a+b", "0", 4, [x], torch.empty((), dtype=torch.int32))
    offs = torch.tensor([0, 4, 8])
    with pytest.raises(hm.InvalidError, match="2 are written"):
        hm.reduce_segmented(r, "a+b", "0", offs, 8, [x], torch.empty(1))
    with pytest.raises(hm.MismatchError, match="int64"):
        hm.reduce_segmented(r, "a+b", "0", offs.to(torch.int32), 8, [x], torch.empty(2))
    with pytest.raises(hm.InvalidError, match="nseg"):
        hm.reduce_segmented(r, "a+b", "0", offs.reshape(1, 3), 8, [x], torch.empty(2))
