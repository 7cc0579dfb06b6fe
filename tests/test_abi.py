"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "hbl.h")).read()
    return sorted(set(re.findall(r"\b(hbl_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(hbl):
    decl = declared_symbols()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(hbl.lib, name), name


def test_version(hbl):
    assert "gfx950" in hbl.version()


def _d6(*v):
    return (C.c_double * 6)(*(v or (0.0,) * 6))


BAD = C.c_void_p(0x1000)      # 16-byte aligned; never dereferenced: validation rejects first


@pytest.mark.parametrize("args,frag", [
    ((None, 10, 10), "NULL bunch"),
    ((BAD, -1, 10), "n = -1"),
    ((BAD, 10, 8), "ld = 8 < n"),
    ((BAD, 10, 11), "must be even"),
    ((C.c_void_p(0x1008), 10, 10), "16-byte aligned"),
])
def test_fill_rejects_bad_bunch(hbl, args, frag):
    rc = hbl.lib.hbl_bunch_fill_gaussian(*args, 1, _d6(), _d6(), 0, None)
    assert rc == hbl.HBL_EINVAL
    assert frag in hbl.lib.hbl_last_error().decode()


def test_fill_rejects_bad_sigma(hbl):
    rc = hbl.lib.hbl_bunch_fill_gaussian(BAD, 10, 10, 1, _d6(), _d6(1, 1, 1, -1, 1, 1), 0, None)
    assert rc == hbl.HBL_EINVAL and "sigma" in hbl.lib.hbl_last_error().decode()
    rc = hbl.lib.hbl_bunch_fill_gaussian(BAD, 10, 10, 1, _d6(float("nan"), 0, 0, 0, 0, 0), _d6(), 0, None)
    assert rc == hbl.HBL_EINVAL


def _lat(hbl, elems, gamma=1957.0):
    arr = (hbl.Element * len(elems))(*elems)
    h = C.c_void_p()
    ref = hbl.Ref(hbl.MEC2_MEV, gamma, 0.0)
    return hbl.lib.hbl_lattice_create(arr, len(elems), C.byref(ref), C.byref(h))


@pytest.mark.parametrize("el,frag", [
    (dict(kind=99), "unknown element kind"),
    (dict(kind=4, f=0.0), "f must be finite and nonzero"),
    (dict(kind=1, L=float("inf")), "finite"),
    (dict(kind=2, L=1.0, k=float("nan")), "finite"),
    (dict(kind=3, L=0.0, angle=0.1), "nonzero length"),
    (dict(kind=5, L=0.3, nsub=10), "linear elements only"),
    (dict(kind=1, L=1.0, chromatic=1), "quads and thin lenses only"),
    (dict(kind=2, L=1.0, k=1.0, chromatic=2), "chromatic must be 0 or 1"),
    (dict(kind=2, L=1.0, k=1.0, chirp=1.0), "stages only"),
    (dict(kind=4, f=1.0, reserved=1), "reserved"),
])
def test_lattice_rejects_bad_elements(hbl, el, frag):
    rc = _lat(hbl, [hbl.Element(**el)])
    assert rc == hbl.HBL_EINVAL
    assert frag in hbl.lib.hbl_last_error().decode()


def test_lattice_rejects_bad_reference(hbl):
    assert _lat(hbl, [hbl.Element(kind=1, L=1.0)], gamma=1.0) == hbl.HBL_EINVAL
    assert _lat(hbl, [hbl.Element(kind=1, L=1.0)], gamma=float("nan")) == hbl.HBL_EINVAL


@pytest.mark.parametrize("st,frag", [
    (dict(kind=1, L=0.3, nsub=10), "not a stage"),
    (dict(kind=5, L=0.3, nsub=0), "nsub"),
    (dict(kind=5, L=-0.3, nsub=10), "L must be"),
    (dict(kind=5, L=0.3, nsub=10, n0_m3=-1.0), "n0"),
    (dict(kind=5, L=0.3, nsub=10, dE_MeV=-2000.0), "exit gamma"),
    (dict(kind=5, L=0.3, nsub=10, chirp=float("nan")), "chirp"),
    (dict(kind=5, L=0.3, nsub=10, chromatic=1), "chromatic/reserved"),
])
def test_stage_rejects_bad_parameters(hbl, st, frag):
    el = hbl.Element(**st)
    ref = hbl.Ref.from_energy(1000.0)
    rc = hbl.lib.hbl_apply_stage(BAD, 10, 10, C.byref(el), C.byref(ref), None, 0, None)
    assert rc == hbl.HBL_EINVAL and frag in hbl.lib.hbl_last_error().decode()
    assert ref.gamma == 1000.0 / hbl.MEC2_MEV          # rejected call has no effect


def test_stage_rejects_overlapping_record(hbl):
    el = hbl.Element(kind=5, L=0.3, nsub=10, n0_m3=1e23, dE_MeV=100.0)
    ref = hbl.Ref.from_energy(1000.0)
    rc = hbl.lib.hbl_apply_stage(BAD, 10, 10, C.byref(el), C.byref(ref), C.c_void_p(0x1000 + 160), 10, None)
    assert rc == hbl.HBL_EINVAL and "overlaps" in hbl.lib.hbl_last_error().decode()


def test_moments_and_compare_reject(hbl):
    m, c = _d6(), (C.c_double * 21)()
    assert hbl.lib.hbl_moments(BAD, 0, 0, m, c, None) == hbl.HBL_EINVAL
    assert hbl.lib.hbl_moments(BAD, 4, 4, None, c, None) == hbl.HBL_EINVAL
    r, e = _d6(), (C.c_double * 3)()
    assert hbl.lib.hbl_compare(BAD, None, 4, 4, r, m, e, None) == hbl.HBL_EINVAL
    for args, frag in (((BAD, 0, 0, BAD), "n >= 1"), ((BAD, 4, 4, None), "output pointer"),
                       ((BAD, 4, 4, C.c_void_p(0x1004)), "output pointer"), ((BAD, 4, 3, BAD), "ld")):
        assert hbl.lib.hbl_moments_async_noalloc(*args, None) == hbl.HBL_EINVAL
        assert frag in hbl.lib.hbl_last_error().decode()


def test_emittances_host_only(hbl):
    cov = [0.0] * 21
    cov[0] = 4.0       # <x x>
    cov[3] = 1.0       # <x px>
    cov[15] = 1.0      # <px px>
    e = hbl.emittances(cov)
    assert abs(e[0] - 3.0 ** 0.5) < 1e-15 and e[1] == 0.0
    bad = list(cov)
    bad[0] = float("inf")
    with pytest.raises(hbl.HblError):
        hbl.emittances(bad)


@pytest.mark.parametrize("shape,frag", [
    ((6, 7, 3, 6), "width 7"),
    ((6, 1025, 3, 6), "width 1025"),
    ((6, 700, 0, 6), "hidden 0"),
    ((6, 700, 8, 6), "hidden 8"),
    ((5, 700, 3, 6), "n_in and n_out"),
    ((6, 700, 3, 4), "n_in and n_out"),
])
def test_prelu_create_rejects_bad_shapes(hbl, shape, frag):
    h = C.c_void_p()
    rc = hbl.lib.hbl_prelu_create(C.byref(hbl.MlpShape(*shape)), 0, C.byref(h))
    assert rc == hbl.HBL_EINVAL and frag in hbl.lib.hbl_last_error().decode()
    assert h.value is None


def test_prelu_calls_reject_null_handles(hbl):
    n = C.c_int64()
    assert hbl.lib.hbl_prelu_num_params(None, C.byref(n)) == hbl.HBL_EINVAL
    assert hbl.lib.hbl_prelu_apply(BAD, 10, 10, None, None, None) == hbl.HBL_EINVAL
    assert hbl.lib.hbl_prelu_apply(BAD, 10, 9, None, None, None) == hbl.HBL_EINVAL
    assert hbl.lib.hbl_prelu_set_norm(None, (C.c_double * 24)()) == hbl.HBL_EINVAL


def test_prelu_load_rejects_missing_and_foreign_files(hbl, tmp_path):
    h = C.c_void_p()
    assert hbl.lib.hbl_prelu_load(str(tmp_path / "none.bin").encode(), C.byref(h)) == hbl.HBL_EIO
    p = tmp_path / "junk.bin"
    p.write_bytes(b"not a network file" * 20)
    assert hbl.lib.hbl_prelu_load(str(p).encode(), C.byref(h)) == hbl.HBL_EIO
    assert "not a PReLU network file" in hbl.lib.hbl_last_error().decode()
