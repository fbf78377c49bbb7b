"""The C-ABI library loads, exports every symbol include/lattice.h declares and
validates its arguments before touching a device (no compute calls here)."""
import ctypes as C
import math
import os

import pytest

from paper_2102_01031_amd import lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_built_and_exports_header_symbols():
    lib = L.lib()
    names = L.declared_symbols()
    assert {"lattice_init", "lattice_step", "lattice_energy", "lattice_destroy", "lattice_sync"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.lattice_version()


def test_no_oracle_in_product_path():
    pkg = os.path.join(ROOT, "paper_2102_01031_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "lattice_oracle" not in txt, f


def _fields(nf=1, u1=False):
    f = L.LatFields()
    for i in range(2):
        f.phi[i] = 0x10000 + 0x1000 * i
        f.pi[i] = 0x20000 + 0x1000 * i
    if u1:
        for i in range(3):
            f.A[i] = 0x30000 + 0x1000 * i
            f.piA[i] = 0x40000 + 0x1000 * i
    return f


def _init(params, fields):
    ctx = C.c_void_p()
    rc = L.lib().lattice_init(C.byref(ctx), C.byref(params), C.byref(fields), None)
    return rc, ctx


@pytest.mark.parametrize("kw,code", [
    (dict(N=1, dx=0.5, dt=0.01), L.LAT_EINVAL),
    (dict(N=8, dx=0.5, dt=0.3), L.LAT_EINVAL),          # dt/dx above 1/sqrt(3)
    (dict(N=8, dx=-1.0, dt=0.01), L.LAT_EINVAL),
    (dict(N=8, dx=0.5, dt=0.01, integrator="lf", expansion="self", lf_staggered=1), L.LAT_EINVAL),  # needs b0
    (dict(N=8, dx=0.5, dt=0.01, potential="su2_higgs", integrator="vv2", expansion="fixed", H0=0.1,
          precision="f32"), L.LAT_EUNSUPPORTED),
    (dict(N=8, dx=0.5, dt=0.01, potential="abelian_higgs", precision="f32"), L.LAT_EUNSUPPORTED),
    (dict(N=8, dx=0.5, dt=0.01, integrator="vv2", lf_staggered=1), L.LAT_EINVAL),
])
def test_validation_errors(kw, code):
    p = L.make_params(**kw)
    rc, ctx = _init(p, _fields(2, True))
    assert rc == code
    assert not ctx.value
    assert L.lib().lattice_last_error(None)


def test_integrator_codes():
    """LF, VV2 ... VV10 are codes 0 ... 5; anything else is refused before any device call."""
    assert L.INTEGRATORS == {"lf": 0, "vv2": 1, "vv4": 2, "vv6": 3, "vv8": 4, "vv10": 5}
    p = L.make_params(N=8, dx=0.5, dt=0.01)
    for bad in (6, -1):
        p.integrator = bad
        rc, ctx = _init(p, _fields(1))
        assert rc == L.LAT_EINVAL and not ctx.value


def test_null_and_misaligned_pointers():
    p = L.make_params(N=8, dx=0.5, dt=0.01, potential="phi4_chi2")
    f = _fields(2)
    f.pi[1] = None
    assert _init(p, f)[0] == L.LAT_EINVAL
    f = _fields(2)
    f.phi[1] = 0x10003
    assert _init(p, f)[0] == L.LAT_EINVAL


def test_no_device_here_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = L.make_params(N=8, dx=0.5, dt=0.01, integrator="vv4", expansion="self", potential="phi4_chi2", b0=math.nan)
    rc, ctx = _init(p, _fields(2))
    assert rc == L.LAT_ENODEV
    assert b"GPU" in L.lib().lattice_last_error(None)


def _su2_fields():
    f = L.LatFields()
    for k in range(4):
        f.doublet[k] = 0x50000 + 0x1000 * k
        f.pi_doublet[k] = 0x60000 + 0x1000 * k
    for k in range(12):
        f.U[k] = 0x70000 + 0x1000 * k
    for k in range(9):
        f.E[k] = 0x90000 + 0x1000 * k
    return f


@pytest.mark.parametrize("kw,code", [
    (dict(precision="f32"), L.LAT_EUNSUPPORTED),
    (dict(g=0.0), L.LAT_EINVAL),
    (dict(N=1700), L.LAT_EUNSUPPORTED),        # 8 N^3 >= 2^32: 32-bit offsets
])
def test_su2_validation_errors(kw, code):
    """SU(2) arguments are checked before any device call."""
    base = dict(N=8, dx=0.4, dt=0.02, potential="su2_higgs", g=0.5)
    base.update(kw)
    rc, ctx = _init(L.make_params(**base), _su2_fields())
    assert rc == code, (kw, rc, L.lib().lattice_last_error(None))
    assert not ctx.value


@pytest.mark.parametrize("group,k", [("doublet", 2), ("pi_doublet", 0), ("U", 11), ("E", 4)])
def test_su2_null_and_misaligned_pointers(group, k):
    p = L.make_params(N=8, dx=0.4, dt=0.02, potential="su2_higgs", g=0.5)
    f = _su2_fields()
    getattr(f, group)[k] = None
    assert _init(p, f)[0] == L.LAT_EINVAL
    assert b"SU(2)" in L.lib().lattice_last_error(None)
    f = _su2_fields()
    getattr(f, group)[k] = 0x80004
    assert _init(p, f)[0] == L.LAT_EINVAL


def test_su2_fields_struct_layout():
    """The ctypes mirror of lat_fields: the SU(2) members follow the U(1) ones."""
    assert L.LatFields.doublet.offset == 10 * C.sizeof(C.c_void_p)
    assert L.LatFields.E.offset == (10 + 4 + 4 + 12) * C.sizeof(C.c_void_p)
    assert C.sizeof(L.LatFields) == 39 * C.sizeof(C.c_void_p)


def test_null_context_calls():
    lib = L.lib()
    assert lib.lattice_step(None, 1) == L.LAT_EINVAL
    assert lib.lattice_sync(None) == L.LAT_EINVAL
    e = L.LatEnergies()
    assert lib.lattice_energy(None, C.byref(e)) == L.LAT_EINVAL
    lib.lattice_destroy(None)


def _init_batch(params, sizes, nfields=None):
    n = len(sizes)
    arr = (C.c_int32 * max(n, 1))(*sizes)
    fl = (L.LatFields * max(n, 1))()
    for r in range(n):
        fl[r].phi[0] = 0x10000 + 0x100000 * r
        fl[r].pi[0] = 0x20000 + 0x100000 * r
    ctx = C.c_void_p()
    rc = L.lib().lattice_init_batch(C.byref(ctx), C.byref(params), n if nfields is None else nfields, arr, fl, 0,
                                    None)
    return rc, ctx


@pytest.mark.parametrize("kw,sizes,n,code", [
    (dict(dx=0.5, dt=0.01, integrator="vv2"), [8, 16], None, L.LAT_EUNSUPPORTED),
    (dict(dx=0.5, dt=0.01, potential="phi4_chi2"), [8, 16], None, L.LAT_EUNSUPPORTED),
    (dict(dx=0.5, dt=0.01, integrator="vv4", expansion="self"), [8], None, L.LAT_EUNSUPPORTED),
    (dict(dx=0.5, dt=0.01), [8, 16], 0, L.LAT_EINVAL),
    (dict(dx=0.5, dt=0.01), [8, 1, 16], None, L.LAT_EINVAL),        # a realization with N = 1
    (dict(dx=0.5, dt=0.3), [8], None, L.LAT_EINVAL),                 # dt/dx above 1/sqrt(3)
])
def test_batch_validation_errors(kw, sizes, n, code):
    """Batch contexts: unsupported physics is refused before any device call, and
    a bad realization fails the whole batch with nothing left allocated."""
    p = L.make_params(N=8, **kw)
    rc, ctx = _init_batch(p, sizes, n)
    assert rc == code
    assert not ctx.value
    assert L.lib().lattice_last_error(None)


def test_noalloc_energy_refusals_before_any_device_call():
    """lattice_energy_noalloc validates like lattice_init and refuses lattices
    whose launch needs more block partials than its fixed scratch holds, before
    any device call (fake, aligned pointers)."""
    lib = L.lib()
    out = C.c_void_p(0x50000)
    for kw, code in [
        (dict(N=1, dx=0.5, dt=0.01), L.LAT_EINVAL),
        (dict(N=8, dx=0.5, dt=0.3), L.LAT_EINVAL),
        (dict(N=8, dx=0.5, dt=0.01, potential="abelian_higgs", e=0.5), L.LAT_EUNSUPPORTED),
        # odd N takes 8 x 8 tiles: ceil(1001/8)^2 blocks x 6 sums > 65408
        (dict(N=1001, dx=0.5, dt=0.01, potential="phi4_chi2", q=1.0), L.LAT_EINVAL),
    ]:
        p = L.make_params(**kw)
        rc = lib.lattice_energy_noalloc(C.byref(p), C.byref(_fields(2, True)), out, None)
        assert rc == code, (kw, rc)
        assert lib.lattice_last_error(None)
    p = L.make_params(N=8, dx=0.5, dt=0.01)
    assert lib.lattice_energy_noalloc(C.byref(p), C.byref(_fields(1)), None, None) == L.LAT_EINVAL
    assert lib.lattice_energy_noalloc(C.byref(p), C.byref(_fields(1)), C.c_void_p(0x50004), None) == L.LAT_EINVAL
    msg = lib.lattice_last_error(None).decode()
    assert "output" in msg
