"""Host-side checks of the C ABI (no GPU needed): every symbol that
include/pnce.h declares is exported, and argument validation answers before
any HIP call."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnce.h")
LIB = os.path.join(ROOT, "paper_2206_05506_amd", "libpnce.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pnce_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpnce.so is not built (run python paper_2206_05506_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pnce_create", "pnce_destroy", "pnce_estimate", "pnce_adjoint", "pnce_pack",
              "pnce_estimate_packed", "pnce_refine", "pnce_debias", "pnce_estimate_ls",
              "pnce_get_sequence"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pnce_\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(lib, n)


def test_python_binding_names_match_header():
    sys.path.insert(0, ROOT)
    from paper_2206_05506_amd import _lib
    for n in declared_functions():
        assert hasattr(_lib, n), n
    assert set(_lib.SYMBOLS) == set(declared_functions())


def _create(lib, N, T, L, R):
    h = ctypes.c_void_p()
    lib.pnce_create.argtypes = [ctypes.POINTER(ctypes.c_void_p)] + [ctypes.c_int] * 4
    st = lib.pnce_create(ctypes.byref(h), N, T, L, R)
    return st, h


@pytest.mark.parametrize("N,T,L,R,want", [
    (1000, 4, 16, 16, -2),    # not 2^d - 1
    (1, 1, 1, 1, -2),         # d = 1
    (131071, 1, 1, 1, -2),    # d = 17
    (0, 1, 1, 1, -2),
    (127, 0, 16, 16, -1),
    (127, 4, -1, 16, -1),
    (127, 4, 16, 0, -1),
    (127, 4, 16, 70000, -1),  # R above 65535
    (127, 200, 16, 1, -1),    # T*L > 16 N
    (65535, 16, 4096, 4096, -2),  # one frame beyond 32-bit byte offsets
    (65535, 16, 65535, 100, -2),  # T*L = 16 N: the adjoint's bit stream exceeds LDS
])
def test_create_validates_before_touching_the_device(lib, N, T, L, R, want):
    st, h = _create(lib, N, T, L, R)
    assert st == want
    assert not h.value


def test_create_null_output_pointer(lib):
    lib.pnce_create.argtypes = [ctypes.c_void_p] + [ctypes.c_int] * 4
    assert lib.pnce_create(None, 127, 4, 16, 16) == -1


def test_null_plan_is_rejected_everywhere(lib):
    P = ctypes.c_void_p
    lib.pnce_estimate.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, P,
                                  ctypes.c_double]
    assert lib.pnce_estimate(None, None, None, None, 1, 0, 1.0, None, 0.0) == -1
    lib.pnce_adjoint.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double]
    assert lib.pnce_adjoint(None, None, None, None, None, 1, 0, 1.0, 0.0) == -1
    lib.pnce_refine.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int]
    assert lib.pnce_refine(None, None, None, None, None, 1, 1) == -1
    lib.pnce_refine_noalloc.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int]
    assert lib.pnce_refine_noalloc(None, None, None, None, 1, 1) == -1
    lib.pnce_pack.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int]
    assert lib.pnce_pack(None, None, None, None, None, 1, 1) == -1
    lib.pnce_pack_ws.argtypes = [P, P, P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, P,
                                 ctypes.c_size_t]
    assert lib.pnce_pack_ws(None, None, None, 0, None, None, 1, 1, None, 0) == -1
    lib.pnce_estimate_host.argtypes = [P, P, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, P, ctypes.c_size_t]
    assert lib.pnce_estimate_host(None, None, None, None, 0, None, 1, 1, 1, None, 0) == -1
    lib.pnce_debias.argtypes = [P, P, P, ctypes.c_int]
    assert lib.pnce_debias(None, None, None, 1) == -1
    lib.pnce_estimate_ls.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, P]
    assert lib.pnce_estimate_ls(None, None, None, None, 1, 1, None) == -1
    lib.pnce_destroy.argtypes = [P]
    assert lib.pnce_destroy(None) == 0
    lib.pnce_get_sequence.argtypes = [P, P]
    assert lib.pnce_get_sequence(None, None) == -1


def test_status_strings(lib):
    lib.pnce_status_string.restype = ctypes.c_char_p
    for st in (0, 1, -1, -2, -3, -4):
        assert lib.pnce_status_string(st)
    assert lib.pnce_status_string(99) == b"unknown status"


def test_alloc_fault_hook():
    code = ("import ctypes,sys; l=ctypes.CDLL(sys.argv[1]); h=ctypes.c_void_p();"
            "l.pnce_last_error.restype=ctypes.c_char_p;"
            "st=l.pnce_create(ctypes.byref(h),127,4,16,16);"
            "print(st, l.pnce_last_error().decode())")
    env = dict(os.environ, PNCE_FAULT="alloc")
    out = subprocess.run([sys.executable, "-c", code, LIB], capture_output=True, text=True,
                         env=env, check=True).stdout.split(None, 1)
    assert out[0] == "-3" and "PNCE_FAULT" in out[1]


def _create_ex(lib, N, T, L, R, fb, spacing):
    h = ctypes.c_void_p()
    lib.pnce_create_ex.argtypes = ([ctypes.POINTER(ctypes.c_void_p)] + [ctypes.c_int] * 4 +
                                   [ctypes.c_uint, ctypes.c_int])
    st = lib.pnce_create_ex(ctypes.byref(h), N, T, L, R, fb, spacing)
    return st, h


@pytest.mark.parametrize("N,T,L,fb,spacing", [
    (127, 4, 16, 0, 2),        # unknown spacing
    (127, 8, 16, 0, 1),        # Eq. 8 with T*L > N: blocks overlap (Eq. 7)
    (127, 4, 16, 0x80, 0),     # a tap at or above degree 7
    (63, 4, 8, 0x9, 1),        # x^6 + x^3 + 1: irreducible, not primitive
    (31, 2, 4, 0x3, 0),        # x^5 + x + 1 = (x^2+x+1)(x^3+x^2+1)
])
def test_create_ex_validates_before_touching_the_device(lib, N, T, L, fb, spacing):
    st, h = _create_ex(lib, N, T, L, 4, fb, spacing)
    assert st == -1
    assert not h.value


def test_create_ex_accepts_exactly_the_primitive_polynomials():
    """The library's maximal-length check agrees with the oracle's list for
    every feedback mask of degrees 5 and 6 (accepted masks reach the device
    allocation, which the fault hook fails)."""
    sys.path.insert(0, ROOT)
    import oracle
    want = {d: set(oracle.primitive_masks(d)) for d in (5, 6)}
    code = ("import ctypes,sys; l=ctypes.CDLL(sys.argv[1]); h=ctypes.c_void_p();"
            "l.pnce_create_ex.argtypes=[ctypes.c_void_p]+[ctypes.c_int]*4+[ctypes.c_uint,ctypes.c_int];"
            "print(' '.join(str(l.pnce_create_ex(ctypes.byref(h),(1<<d)-1,2,4,4,m,0))"
            " for d in (5,6) for m in range(1,1<<d)))")
    env = dict(os.environ, PNCE_FAULT="alloc")
    out = subprocess.run([sys.executable, "-c", code, LIB], capture_output=True, text=True,
                         env=env, check=True).stdout.split()
    got = iter(int(x) for x in out)
    for d in (5, 6):
        for m in range(1, 1 << d):
            assert next(got) == (-3 if m in want[d] else -1), (d, m)


def test_lag_and_feedback_queries_reject_null_plan(lib):
    P = ctypes.c_void_p
    lib.pnce_get_lags.argtypes = [P, P]
    assert lib.pnce_get_lags(None, None) == -1
    lib.pnce_get_feedback.argtypes = [P, P]
    assert lib.pnce_get_feedback(None, None) == -1


class _Desc(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("N", ctypes.c_int), ("T", ctypes.c_int),
                ("L", ctypes.c_int), ("y_off", ctypes.c_longlong), ("h_off", ctypes.c_longlong)]


@pytest.mark.parametrize("frames,fmt,want", [
    ([(32, 1000, 4, 16, 0, 0)], 1, -2),          # N not 2^d - 1
    ([(32, 255, 4, 16, 0, 0), (32, 511, 0, 16, 8192, 4096)], 1, -1),   # T = 0 in frame 1
    ([(70000, 255, 4, 16, 0, 0)], 1, -1),        # R above 65535
    ([(32, 255, 4, 16 * 255, 0, 0)], 1, -1),     # T*L > 16 N
    ([(32, 255, 4, 16, 4, 0)], 1, -1),           # y_off not a multiple of 8
    ([(32, 255, 4, 16, -8, 0)], 1, -1),          # negative offset
    ([(32, 255, 4, 16, 0, 0)], 3, -1),           # e4m3 is not a varlen format
    ([], 1, -1),                                 # no frames
])
def test_varlen_create_validates_before_touching_the_device(lib, frames, fmt, want):
    arr = (_Desc * max(1, len(frames)))(*[_Desc(*f) for f in frames])
    h = ctypes.c_void_p()
    lib.pnce_varlen_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int]
    st = lib.pnce_varlen_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(frames),
                                fmt)
    assert st == want
    assert not h.value


def test_more_entry_points_reject_null_plan(lib):
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.pnce_estimate_cp.argtypes = [P, P, P, I, P, I, I, P]
    assert lib.pnce_estimate_cp(None, None, None, 0, None, 1, 1, None) == -1
    lib.pnce_pack_cp.argtypes = [P, P, P, I, P, P, I, I]
    assert lib.pnce_pack_cp(None, None, None, 0, None, None, 1, 1) == -1
    lib.pnce_estimate_packed.argtypes = [P, P, P, P, P, I, I, ctypes.c_double]
    assert lib.pnce_estimate_packed(None, None, None, None, None, 1, 1, 0.0) == -1
    lib.pnce_get_shape.argtypes = [P, P, P, P, P]
    assert lib.pnce_get_shape(None, None, None, None, None) == -1
    for name in ("pnce_varlen_estimate", "pnce_varlen_estimate_each"):
        fn = getattr(lib, name)
        fn.argtypes = [P, P, P, P, P]
        assert fn(None, None, None, None, None) == -1
    lib.pnce_varlen_tune.argtypes = [P, P, P, P, P, I]
    assert lib.pnce_varlen_tune(None, None, None, None, None, 1) == -1
    lib.pnce_varlen_destroy.argtypes = [P]
    assert lib.pnce_varlen_destroy(None) == 0


def _expected_create_status(N, T, L, R, fb, spacing):
    """pnce_create_ex's documented validation, in its order, restated: the
    status a call must return when the device allocation (made only after
    every check passes) fails through the fault hook."""
    import oracle
    if T <= 0 or L <= 0 or R <= 0:
        return -1
    d = next((k for k in range(2, 17) if (1 << k) - 1 == N), None)
    if d is None:
        return -2
    K = T * L
    if K > 16 * N:
        return -1
    if spacing not in (0, 1):
        return -1
    if spacing == 1 and K > N:
        return -1
    if fb >> d:
        return -1
    if fb and oracle.mseq_mask(d, fb) is None:
        return -1
    if R > 65535:
        return -1
    if (R + 32) * (max(N, K) + 1) * 8 >= 1 << 31:
        return -2
    return -3


def test_create_ex_validation_matches_its_documented_rules():
    """400 seeded argument sets (valid and invalid N, T, L, R, feedback masks
    and spacings): every status equals the documented rules restated above,
    and no call leaves a plan behind. Shapes stay far below the LDS limit of
    the bit stream, which has its own test."""
    import random
    sys.path.insert(0, ROOT)
    import oracle
    rnd = random.Random(7)
    cases = []
    for _ in range(400):
        d = rnd.randint(1, 17)
        N = (1 << d) - 1 if rnd.random() < 0.85 else rnd.choice([0, -1, 100, 1000, (1 << d)])
        N = min(N, 32767) if N > 0 and rnd.random() < 0.9 else N
        T = rnd.randint(1, 64) if rnd.random() < 0.9 else rnd.choice([0, -3])
        L = rnd.randint(1, 256) if rnd.random() < 0.9 else 0
        Nn = max(N, 1)
        if T > 0 and L > 0 and T * L > 4 * Nn:      # keep the stream far below the LDS limit
            L = max(1, (4 * Nn) // T)
        r = rnd.random()
        R = (rnd.randint(1, 512) if r < 0.8 else 0 if r < 0.85 else
             rnd.choice([65535, 65536]) if r < 0.93 else rnd.randint(1, 70000))
        dd = next((k for k in range(2, 17) if (1 << k) - 1 == N), 5)
        r = rnd.random()
        if r < 0.55:
            fb = 0
        elif r < 0.75:
            fb = rnd.choice(oracle.primitive_masks(dd)) if dd <= 12 else rnd.randint(1, (1 << dd) - 1)
        elif r < 0.95:
            fb = rnd.randint(1, (1 << dd) - 1)
        else:
            fb = rnd.randint(1 << dd, 1 << 17)
        spacing = rnd.choice([0, 1]) if rnd.random() < 0.9 else rnd.choice([2, -1])
        cases.append((N, T, L, R, fb, spacing))
    code = ("import ctypes,sys,json; l=ctypes.CDLL(sys.argv[1]); "
            "l.pnce_create_ex.argtypes=[ctypes.c_void_p]+[ctypes.c_int]*4+[ctypes.c_uint,ctypes.c_int];"
            "out=[]\n"
            "for N,T,L,R,fb,sp in json.loads(sys.stdin.read()):\n"
            "  h=ctypes.c_void_p(); st=l.pnce_create_ex(ctypes.byref(h),N,T,L,R,fb,sp)\n"
            "  out.append([st, bool(h.value)])\n"
            "print(json.dumps(out))")
    import json
    env = dict(os.environ, PNCE_FAULT="alloc")
    res = subprocess.run([sys.executable, "-c", code, LIB], input=json.dumps(cases),
                         capture_output=True, text=True, env=env, check=True).stdout
    got = json.loads(res)
    seen = set()
    for case, (st, left) in zip(cases, got):
        want = _expected_create_status(*case)
        assert st == want, (case, st, want)
        assert not left, case
        seen.add(want)
    assert seen == {-1, -2, -3}


def _expected_varlen_status(frames, fmt):
    """pnce_varlen_create's documented validation, restated in its order;
    None when every check passes (the call then reaches the device)."""
    if not frames:
        return -1
    if fmt not in (1, 2):
        return -1
    for R, N, T, L, yo, ho in frames:
        if not any((1 << k) - 1 == N for k in range(2, 17)):
            return -2
        if R <= 0 or T <= 0 or L <= 0 or R > 65535 or T * L > 16 * N:
            return -1
        if (R + 32) * 2 * (N + 1) * 2 >= 1 << 31:
            return -2
        if yo < 0 or ho < 0 or yo % 8:
            return -1
    return None


def test_varlen_create_validation_matches_its_documented_rules():
    """300 seeded frame lists (one to four frames, each field now and then
    invalid) and formats: every refused list gets the documented status and
    leaves no plan; an accepted list either builds a plan (on a GPU, then
    destroyed) or fails at the device query (PNCE_E_HIP, here)."""
    import json
    import random
    rnd = random.Random(11)
    cases = []
    for _ in range(300):
        frames = []
        for _ in range(rnd.randint(1, 4) if rnd.random() < 0.95 else 0):
            d = rnd.randint(2, 12)
            N = (1 << d) - 1 if rnd.random() < 0.93 else rnd.choice([0, 100, 1 << d])
            R = rnd.randint(1, 96) if rnd.random() < 0.93 else rnd.choice([0, 65536, 40000])
            T = rnd.randint(1, 16) if rnd.random() < 0.95 else 0
            L = rnd.randint(1, 64) if rnd.random() < 0.95 else rnd.choice([0, 16 * max(N, 1)])
            yo = 8 * rnd.randint(0, 1000) if rnd.random() < 0.93 else rnd.choice([-8, 4, 3])
            ho = rnd.randint(0, 1000) if rnd.random() < 0.97 else -1
            frames.append((R, N, T, L, yo, ho))
        fmt = rnd.choice([1, 2]) if rnd.random() < 0.93 else rnd.choice([0, 3])
        cases.append((frames, fmt))
    code = ("import ctypes,sys,json\n"
            "class D(ctypes.Structure):\n"
            "  _fields_=[('R',ctypes.c_int),('N',ctypes.c_int),('T',ctypes.c_int),('L',ctypes.c_int),"
            "('y_off',ctypes.c_longlong),('h_off',ctypes.c_longlong)]\n"
            "l=ctypes.CDLL(sys.argv[1])\n"
            "l.pnce_varlen_create.argtypes=[ctypes.c_void_p,ctypes.c_void_p,ctypes.c_int,ctypes.c_int]\n"
            "l.pnce_varlen_destroy.argtypes=[ctypes.c_void_p]\n"
            "out=[]\n"
            "for frames,fmt in json.loads(sys.stdin.read()):\n"
            "  arr=(D*max(1,len(frames)))(*[D(*f) for f in frames]); h=ctypes.c_void_p()\n"
            "  st=l.pnce_varlen_create(ctypes.byref(h),ctypes.cast(arr,ctypes.c_void_p),len(frames),fmt)\n"
            "  left=bool(h.value)\n"
            "  if left: l.pnce_varlen_destroy(h)\n"
            "  out.append([st,left])\n"
            "print(json.dumps(out))")
    res = subprocess.run([sys.executable, "-c", code, LIB], input=json.dumps(cases),
                         capture_output=True, text=True, check=True).stdout
    seen = set()
    for (frames, fmt), (st, left) in zip(cases, json.loads(res)):
        want = _expected_varlen_status(frames, fmt)
        if want is None:
            assert st in (0, 1, -4), (frames, fmt, st)
            assert left == (st >= 0)
        else:
            assert st == want, (frames, fmt, st, want)
            assert not left
        seen.add(want)
    assert {-1, -2, None} <= seen
