"""Host-side checks of the C ABI: libkfac.so loads without a GPU, exports every symbol
declared in include/kfac.h, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kfac.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(kfac_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2206_15397_amd import _lib
    if not os.path.exists(_lib.library_path()):
        from paper_2206_15397_amd import build
        build.build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    from paper_2206_15397_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_status_strings(L):
    assert L.kfac_status_string(0) == b"ok"
    assert b"invalid" in L.kfac_status_string(1)
    assert b"workspace" in L.kfac_status_string(2)
    assert L.kfac_build_info().startswith(b"libkfac gfx950")


P = ctypes.c_void_p
FAKE = P(0x10000)   # never dereferenced: validation fails first


def test_ea_update_validation(L):
    ok_args = dict(F=FAKE, d=5, ldf=5, X=FAKE, xt=0, n=3, d_in=4, ldx=4, ones=1, rho=0.95, scale=1 / 3,
                   Fb=P(0), ldfb=0, ws=P(0), wsb=0, st=P(0))

    def call(**kw):
        a = dict(ok_args); a.update(kw)
        return L.kfac_ea_update(a["F"], a["d"], a["ldf"], a["X"], a["xt"], a["n"], a["d_in"], a["ldx"],
                                a["ones"], a["rho"], a["scale"], a["Fb"], a["ldfb"], a["ws"], a["wsb"], a["st"])
    assert call(F=P(0)) == 1
    assert call(d=0) == 1
    assert call(ldf=4) == 1
    assert call(d_in=5) == 1                 # d != d_in + ones
    assert call(ldx=3) == 1
    assert call(rho=1.0) == 1
    assert call(rho=-0.1) == 1
    assert call(scale=0.0) == 1
    assert call(xt=7) == 1
    assert call(Fb=FAKE, ldfb=4) == 1
    assert call(X=P(0)) == 1


def test_rand_eig_validation(L):
    ws = L.kfac_rand_eig_workspace(100, 10, 5, 1, 0, 0)
    assert ws > 0
    assert L.kfac_rand_eig_workspace(100, 101, 5, 1, 0, 0) == 0

    def call(**kw):
        a = dict(F=FAKE, d=100, ldf=100, Fb=P(0), ldfb=0, r=10, p=5, q=1, seed=0, sid=0, inv=0, v=0, prec=0,
                 U=FAKE, ldu=10, D=FAKE, ws=FAKE, wsb=ws, st=FAKE, s=P(0))
        a.update(kw)
        return L.kfac_rand_eig(a["F"], a["d"], a["ldf"], a["Fb"], a["ldfb"], a["r"], a["p"], a["q"], a["seed"],
                               a["sid"], a["inv"], a["v"], a["prec"], a["U"], a["ldu"], a["D"], a["ws"],
                               a["wsb"], a["st"], a["s"])
    assert call(r=0) == 1
    assert call(r=101) == 1
    assert call(p=-1) == 1
    assert call(q=17) == 1
    assert call(ldu=9) == 1
    assert call(ldf=99) == 1
    assert call(st=P(0)) == 1
    assert call(prec=1) == 1                 # bf16 sketch without a bf16 copy of F
    assert call(wsb=ws - 1) == 2
    assert call(v=2) == 1                    # unknown variant
    assert call(r=400, p=200, d=1000, ldf=1000, ldu=400) == 4   # sketch wider than supported


def test_rand_eig_noalloc_validation(L):
    # validation and the scratch-size check happen on the host, before any device call
    def call(**kw):
        a = dict(F=FAKE, d=100, ldf=100, Fb=P(0), ldfb=0, r=10, p=5, q=1, v=0, prec=0, U=FAKE, ldu=10, D=FAKE,
                 st=FAKE)
        a.update(kw)
        return L.kfac_rand_eig_noalloc(a["F"], a["d"], a["ldf"], a["Fb"], a["ldfb"], a["r"], a["p"], a["q"], 0,
                                       0, 0, a["v"], a["prec"], a["U"], a["ldu"], a["D"], a["st"], P(0))
    assert call(r=0) == 1
    assert call(r=101) == 1
    assert call(p=-1) == 1
    from paper_2206_15397_amd import _lib
    big = L.kfac_rand_eig_workspace(16384, 256, 16, 2, 0, 1)
    assert big > _lib.NOALLOC_SCRATCH_BYTES
    assert call(d=16384, ldf=16384, Fb=FAKE, ldfb=16384, r=256, p=16, q=2, prec=1, ldu=256) == _lib.KFAC_ESCRATCH
    assert b"scratch" in L.kfac_status_string(_lib.KFAC_ESCRATCH)


def test_conv_entry_points_validation(L):
    from paper_2206_15397_amd import _lib
    g = _lib.ConvGeom(2, 8, 8, 16, 3, 3, 1, 1)
    d = 9 * 16 + 1
    assert L.kfac_conv_ea_update_workspace(d, ctypes.byref(g)) >= 0

    def ea(geom=g, dd=d, ones=1, rho=0.9, F=FAKE, x=FAKE):
        return L.kfac_conv_ea_update(F, dd, dd, x, ctypes.byref(geom), ones, rho, 0.01, P(0), 0, P(0), 0, P(0))
    assert ea(dd=d - 1) == 1                                   # d != kh kw C + ones
    assert ea(ones=0) == 1
    assert ea(rho=1.0) == 1
    assert ea(F=P(0)) == 1
    assert ea(geom=_lib.ConvGeom(2, 2, 2, 16, 3, 3, 0, 1), dd=d) == 1      # empty output
    assert ea(geom=_lib.ConvGeom(2, 8, 8, 16, 3, 3, 1, 0), dd=d) == 1      # stride 0
    assert ea(geom=_lib.ConvGeom(2, 8, 8, 16, 3, 3, -1, 1), dd=d) == 1     # negative padding

    def bw(lddw=d, c_out=8, Gam=P(0), ws=P(0), wsb=0):
        return L.kfac_conv_backward_weight(FAKE, c_out, FAKE, ctypes.byref(g), FAKE, lddw, 1, Gam, 8, P(0), 8, 0.9,
                                           0.5, ws, wsb, P(0))
    assert bw(lddw=d - 1) == 1
    assert bw(c_out=0) == 1
    # K slices: positions n = 2 * 8 * 8 = 128 give one slice (no workspace); a large input asks for
    # slices, and a short non-null workspace is refused before anything is enqueued
    assert L.kfac_conv_backward_weight_workspace(8, ctypes.byref(g), 1) == 0
    gb = _lib.ConvGeom(128, 32, 32, 64, 3, 3, 1, 1)
    need = L.kfac_conv_backward_weight_workspace(64, ctypes.byref(gb), 1)
    assert need > 0 and need % (128 * 128 * 4) == 0
    assert L.kfac_conv_backward_weight_workspace(0, ctypes.byref(gb), 1) == 0
    short = L.kfac_conv_backward_weight(FAKE, 64, FAKE, ctypes.byref(gb), FAKE, 9 * 64 + 1, 1, P(0), 64, P(0), 64,
                                        0.9, 0.5, FAKE, need - 1, P(0))
    assert short == _lib.KFAC_EWORKSPACE


def test_precondition_validation(L):
    ws = L.kfac_precondition_workspace(8, 9, 3, 2)
    assert ws > 0

    def call(**kw):
        a = dict(J=FAKE, dg=8, da=9, ldj=9, Ua=FAKE, ldua=3, Da=FAKE, ra=3, Ug=FAKE, ldug=2, Dg=FAKE, rg=2,
                 lam=0.1, S=P(0x20000), lds=9, ws=FAKE, wsb=ws, s=P(0))
        a.update(kw)
        return L.kfac_precondition(a["J"], a["dg"], a["da"], a["ldj"], a["Ua"], a["ldua"], a["Da"], a["ra"],
                                   a["Ug"], a["ldug"], a["Dg"], a["rg"], a["lam"], a["S"], a["lds"], a["ws"],
                                   a["wsb"], a["s"])
    assert call(lam=0.0) == 1
    assert call(lam=-1.0) == 1
    assert call(ra=10) == 1
    assert call(ldua=2) == 1
    assert call(S=FAKE) == 1                 # aliasing J
    assert call(lds=8) == 1
    assert call(wsb=ws - 1) == 2


def test_fill_identity_and_omega_validation(L):
    assert L.kfac_fill_identity(P(0), 4, 4, P(0)) == 1
    assert L.kfac_fill_identity(FAKE, 4, 3, P(0)) == 1
    assert L.kfac_gaussian_omega(P(0), 4, 4, 4, 0, 0, 0, P(0), P(0)) == 1
    assert L.kfac_gaussian_omega(FAKE, 4, 4, 3, 0, 0, 0, P(0), P(0)) == 1


def test_workspace_queries_monotone(L):
    a = L.kfac_rand_eig_workspace(1000, 64, 16, 1, 0, 0)
    b = L.kfac_rand_eig_workspace(2000, 64, 16, 1, 0, 0)
    c = L.kfac_rand_eig_workspace(2000, 64, 16, 1, 0, 1)
    assert 0 < a < b < c
    assert L.kfac_ea_update_workspace(577, 131072) > 0
    assert L.kfac_ea_update_workspace(16384, 512) == 0   # enough tiles without split-K
