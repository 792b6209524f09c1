"""The C ABI library loads and exports every function include/lbm.h declares;
host-only calls validate their arguments.  No GPU needed (no kernel runs)."""
import ctypes as C
import os
import re

import pytest

from paper_1809_06735_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return re.findall(r"^LBM_API\s+[\w\s\*]+?\b(lbm3?_\w+)\s*\(", src, flags=re.M)


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("lbm_init", "lbm_step", "lbm_moments", "lbm_subvolume_balance", "lbm3_init",
                 "lbm3_step", "lbm3_moments", "lbm3_subvolume_balance"):
        assert core in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # every declared function has a ctypes signature in the binding, and vice versa
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_version_and_strerror():
    lib = L.load()
    assert b"gfx950" in lib.lbm_version()
    assert lib.lbm_strerror(L.LBM_E_DIVERGED) == b"simulation diverged"
    assert lib.lbm_strerror(12345) == b"unknown status"


def cfg(**kw):
    base = dict(nx=64, ny=64, dtype=L.LBM_F32, has_force=0, with_balance=0, layout=0,
                tau=0.6, drag_alpha=0.0, stream=None)
    base.update(kw)
    return L.Config(**base)


def test_workspace_bytes_and_validation():
    lib = L.load()
    n = C.c_size_t()
    assert lib.lbm_workspace_bytes(C.byref(cfg()), C.byref(n)) == L.LBM_OK
    pops = 2 * 9 * 64 * 64 * 4
    assert n.value >= pops
    n64 = C.c_size_t()
    lib.lbm_workspace_bytes(C.byref(cfg(dtype=L.LBM_F64)), C.byref(n64))
    assert n64.value > n.value
    nb = C.c_size_t()
    lib.lbm_workspace_bytes(C.byref(cfg(with_balance=1)), C.byref(nb))
    assert nb.value > n.value + 13 * 65 * 65 * 8
    bad = [cfg(tau=0.5), cfg(tau=float("nan")), cfg(nx=8), cfg(dtype=7), cfg(drag_alpha=-1.0),
           cfg(has_force=2), cfg(layout=2), cfg(ny=70000)]
    for c in bad:
        assert lib.lbm_workspace_bytes(C.byref(c), C.byref(n)) == L.LBM_E_INVALID
        assert lib.lbm_last_error()
    assert lib.lbm_workspace_bytes(None, C.byref(n)) == L.LBM_E_INVALID


def test_init_rejects_bad_arguments_before_touching_the_device():
    lib = L.load()
    h = C.c_void_p()
    # NULL workspace / misaligned workspace / NULL fields: rejected on the host
    assert lib.lbm_init(C.byref(cfg()), None, 0, None, None, None, None, None, C.byref(h)) == L.LBM_E_INVALID
    assert lib.lbm_init(C.byref(cfg()), C.c_void_p(8), 1 << 30, C.c_void_p(256), C.c_void_p(256),
                        C.c_void_p(256), None, None, C.byref(h)) == L.LBM_E_INVALID
    assert lib.lbm_init(C.byref(cfg()), C.c_void_p(256), 16, C.c_void_p(256), C.c_void_p(256),
                        C.c_void_p(256), None, None, C.byref(h)) == L.LBM_E_NOMEM
    assert lib.lbm_init(C.byref(cfg(has_force=1)), C.c_void_p(256), 1 << 30, C.c_void_p(256),
                        C.c_void_p(256), C.c_void_p(256), None, None, C.byref(h)) == L.LBM_E_INVALID
    assert lib.lbm_step(None, 1) == L.LBM_E_INVALID
    assert lib.lbm_destroy(None) == L.LBM_OK


def test_balance_workspace_and_adjoint_validation():
    lib = L.load()
    n = C.c_size_t()
    assert lib.lbm_balance_workspace_bytes(64, 64, C.byref(n)) == L.LBM_OK
    assert n.value >= (13 + 8) * 64 * 64 * 8 + 13 * 65 * 65 * 8
    assert lib.lbm_balance_workspace_bytes(8, 64, C.byref(n)) == L.LBM_E_INVALID
    # the window walks address the prefix tables with 32-bit element offsets:
    # 13 (nx + 1)(ny + 1) must stay below 2^32 (18175^2 fits, 18176^2 does not)
    assert 13 * 18176 * 18176 < 2 ** 32 <= 13 * 18177 * 18177
    assert lib.lbm_balance_workspace_bytes(18175, 18175, C.byref(n)) == L.LBM_OK
    assert lib.lbm_balance_workspace_bytes(18176, 18176, C.byref(n)) == L.LBM_E_UNSUPPORTED
    assert b"2^32" in lib.lbm_last_error()
    assert lib.lbm_balance_workspace_bytes(65536, 6000, C.byref(n)) == L.LBM_E_UNSUPPORTED
    assert lib.lbm_balance_workspace_bytes(65536, 5000, C.byref(n)) == L.LBM_OK
    # a handle with the balance refuses such a grid; without it the step alone is fine
    assert lib.lbm_workspace_bytes(C.byref(cfg(nx=20000, ny=20000, with_balance=1)),
                                   C.byref(n)) == L.LBM_E_UNSUPPORTED
    assert lib.lbm_workspace_bytes(C.byref(cfg(nx=20000, ny=20000)), C.byref(n)) == L.LBM_OK
    # the allocation-free balance refuses grids beyond its static scratch (host check, before
    # anything touches a device) and validates its arguments like lbm_balance_fields
    inp = L.BalanceInput()
    for k in range(3):
        inp.rho[k] = inp.ux[k] = inp.uy[k] = 256
    inp.nx, inp.ny, inp.nu = 640, 640, 0.001
    sz = (C.c_int32 * 1)(8)
    st = (L.BalanceStats * 1)()
    assert lib.lbm_balance_fields_noalloc(C.byref(inp), sz, 1, st, None, None, 0, None, None) == L.LBM_E_NOMEM
    assert b"scratch" in lib.lbm_last_error()
    inp.nx = inp.ny = 64
    inp.rho[1] = None
    assert lib.lbm_balance_fields_noalloc(C.byref(inp), sz, 1, st, None, None, 0, None, None) == L.LBM_E_INVALID
    assert lib.lbm_balance_fields_noalloc(None, sz, 1, st, None, None, 0, None, None) == L.LBM_E_INVALID
    assert lib.lbm_copy(None, None, 16, None) == L.LBM_E_INVALID
    assert lib.lbm_copy(C.c_void_p(256), C.c_void_p(512), 15, None) == L.LBM_E_INVALID


def test_exact_difference_config_validation():
    """The paper's forced set-up: scheme, damping and shell checks happen on the host."""
    lib = L.load()
    n = C.c_size_t()
    edm = dict(force_scheme=L.LBM_FORCE_EDM)
    ok = [cfg(**edm), cfg(has_force=1, **edm),
          cfg(damp_f0=1e-5, damp_kmin=1.0, damp_kmax=2.0, **edm),
          cfg(damp_f0=1e-5, damp_kmin=0.5, damp_kmax=4.0, **edm)]
    for c in ok:
        assert lib.lbm_workspace_bytes(C.byref(c), C.byref(n)) == L.LBM_OK, lib.lbm_last_error()
    plain = C.c_size_t()
    lib.lbm_workspace_bytes(C.byref(cfg(**edm)), C.byref(plain))
    damped = C.c_size_t()
    lib.lbm_workspace_bytes(C.byref(ok[2]), C.byref(damped))
    assert damped.value > plain.value  # tables, partials and row coefficients
    bad = [cfg(force_scheme=2), cfg(collision=2),
           cfg(damp_f0=1e-5),                                   # damping needs the EDM scheme
           cfg(damp_f0=-1.0, **edm), cfg(damp_f0=float("inf"), **edm),
           cfg(damp_f0=1e-5, damp_kmin=0.0, damp_kmax=2.0, **edm),
           cfg(damp_f0=1e-5, damp_kmin=3.0, damp_kmax=2.0, **edm),
           cfg(damp_f0=1e-5, damp_kmin=1.0, damp_kmax=5.0, **edm),  # beyond |k| = 4
           cfg(damp_f0=1e-5, damp_kmin=1.2, damp_kmax=1.3, **edm)]  # no integer vector
    for c in bad:
        assert lib.lbm_workspace_bytes(C.byref(c), C.byref(n)) == L.LBM_E_INVALID, (
            c.force_scheme, c.damp_f0, c.damp_kmin, c.damp_kmax)
        assert lib.lbm_last_error()
    # drag is a Guo-scheme option; a batch runs the Guo step only
    assert lib.lbm_workspace_bytes(C.byref(cfg(drag_alpha=1e-3, **edm)), C.byref(n)) == L.LBM_E_UNSUPPORTED
    cs = (L.Config * 2)(cfg(), cfg(**edm))
    assert lib.lbm_batch_workspace_bytes(cs, 2, C.byref(n)) == L.LBM_E_UNSUPPORTED
    # the entropic collision: unforced only, not in a batch
    ent = dict(collision=L.LBM_COLLISION_ENTROPIC)
    assert lib.lbm_workspace_bytes(C.byref(cfg(**ent)), C.byref(n)) == L.LBM_OK
    for extra in (dict(has_force=1), dict(drag_alpha=1e-3), dict(force_scheme=L.LBM_FORCE_EDM)):
        assert lib.lbm_workspace_bytes(C.byref(cfg(**ent, **extra)), C.byref(n)) == L.LBM_E_UNSUPPORTED
    cs = (L.Config * 2)(cfg(), cfg(**ent))
    assert lib.lbm_batch_workspace_bytes(cs, 2, C.byref(n)) == L.LBM_E_UNSUPPORTED
    # the exact-difference step takes single-step shapes with one site per thread
    assert lib.lbm_set_tuned_tile(C.byref(cfg(**edm)), C.byref(L.Tile(256, 1, 1, 64, 0, 2, 0))) == L.LBM_E_INVALID
    assert lib.lbm_set_tuned_tile(C.byref(cfg(**edm)), C.byref(L.Tile(64, 4, 2, 1, 0, 1, 0))) == L.LBM_E_INVALID


def test_3d_config_validation():
    """lbm3_workspace_bytes and lbm3_init validate the 3D configuration on the host; a D3Q27
    handle holds 27 populations per site."""
    lib = L.load()

    def c3(**kw):
        base = dict(nx=32, ny=24, nz=16, dtype=L.LBM_F32, has_force=0, with_balance=0, tau=0.6, stream=None)
        base.update(kw)
        return L.Config3(**base)

    n = C.c_size_t()
    assert lib.lbm3_workspace_bytes(C.byref(c3()), C.byref(n)) == L.LBM_OK
    plane = 32 * 24 * 16
    assert n.value >= 2 * 19 * plane * 4
    n64, nb, nf = C.c_size_t(), C.c_size_t(), C.c_size_t()
    lib.lbm3_workspace_bytes(C.byref(c3(dtype=L.LBM_F64)), C.byref(n64))
    lib.lbm3_workspace_bytes(C.byref(c3(with_balance=1)), C.byref(nb))
    lib.lbm3_workspace_bytes(C.byref(c3(has_force=1)), C.byref(nf))
    assert n64.value > n.value and nb.value > n.value + 14 * plane * 8 and nf.value > n.value
    n27 = C.c_size_t()
    assert lib.lbm3_workspace_bytes(C.byref(c3(lattice=1)), C.byref(n27)) == L.LBM_OK
    assert n27.value - n.value >= 2 * 8 * plane * 4
    for bad in (dict(nx=8), dict(nz=5000), dict(dtype=7), dict(tau=0.5), dict(tau=float("nan")),
                dict(has_force=2), dict(with_balance=-1), dict(lattice=2), dict(lattice=-1)):
        assert lib.lbm3_workspace_bytes(C.byref(c3(**bad)), C.byref(n)) == L.LBM_E_INVALID, bad
    assert lib.lbm3_workspace_bytes(None, C.byref(n)) == L.LBM_E_INVALID
    h = C.c_void_p()
    # invalid arguments are rejected before anything touches the device
    assert lib.lbm3_init(C.byref(c3()), None, 0, None, None, None, None, None, None, None,
                         C.byref(h)) == L.LBM_E_INVALID
    assert lib.lbm3_step(None, 1) == L.LBM_E_INVALID
    assert lib.lbm3_destroy(None) == L.LBM_OK


def test_tuned_shape_cache_file_round_trip(tmp_path):
    """lbm_set_tuned_tile writes the process table to LBM_TUNE_CACHE (one line per grid and
    scheme, the eight shape fields including halo) and a new process reads it back (a second
    store from that process keeps the first line).  Host calls only."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    code = (
        "import ctypes as C, sys\n"
        "from paper_1809_06735_amd import _lib as L\n"
        "lib = L.load()\n"
        "cfg = L.Config(nx=%d, ny=256, dtype=L.LBM_F32, has_force=1, with_balance=0, layout=1, tau=0.6,"
        " drag_alpha=1e-3, stream=None)\n"
        "t = L.Tile(%s)\n"
        "sys.exit(lib.lbm_set_tuned_tile(C.byref(cfg), C.byref(t)))\n")
    env = dict(os.environ, LBM_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code % (512, "256, 1, 1, 48, 1, 6, 1, 1")], env=env, cwd=ROOT)
    assert r.returncode == 0
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and lines[0].endswith(": 256 1 1 48 1 6 1 1"), lines
    r = subprocess.run([sys.executable, "-c", code % (1024, "512, 1, 1, 1, 1, 1, 0, 0")], env=env, cwd=ROOT)
    assert r.returncode == 0
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 2 and any(l.endswith(": 256 1 1 48 1 6 1 1") for l in lines), lines
    # an invalid shape is refused and leaves the file alone
    r = subprocess.run([sys.executable, "-c", code % (512, "256, 1, 1, 48, 1, 1, 0, 1")], env=env, cwd=ROOT)
    assert r.returncode != 0 and len(cache.read_text().strip().splitlines()) == 2
