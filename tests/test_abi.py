"""The C ABI library loads, exports every function include/pplbm.h declares, and its host-only
entry points (EOS helpers, validation, error text) work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1412_5170_amd import lbm
    return lbm


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_\w+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_no_undeclared_c_symbol_is_exported(L):
    """Every unmangled function the library exports is one the header declares: helpers next
    to the entry points keep internal linkage."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("needs nm")
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.split()[1:2] == ["T"]}
    plain = {n for n in exported if not n.startswith("_")}
    assert plain - set(declared_functions()) == set(), sorted(plain - set(declared_functions()))


def test_critical_point_matches_oracle(L, thermo):
    rc, Tc, pc = L.eos_critical(L.make_eos(0.5))
    orc, oTc, opc = thermo.critical_point()
    assert Tc == pytest.approx(oTc, rel=1e-13)
    assert rc == pytest.approx(orc, rel=1e-9)      # flat optimum: rho_c is less sharply defined
    assert pc == pytest.approx(opc, rel=1e-12)
    # other constants scale as Tc = 0.37731 a / (b R)
    _, Tc2, _ = L.eos_critical(L.make_eos(0.5, a=2.0, b=3.0, R=0.5))
    assert Tc2 == pytest.approx(Tc * (2.0 / 1.0) * (4.0 / 3.0) / 0.5, rel=1e-13)


@pytest.mark.parametrize("ttc", [0.5, 0.6, 0.8, 0.9])
def test_maxwell_matches_oracle(L, thermo, ttc):
    g, l = L.eos_maxwell(L.make_eos(ttc, K=1 / 49))
    og, ol, _ = thermo.maxwell(ttc)
    assert g == pytest.approx(og, rel=1e-9) and l == pytest.approx(ol, rel=1e-11)


def _create(L, nx=8, ny=8, eos=None, force=None, coll=None, tau=1.0):
    h = ctypes.c_void_p()
    rc = L.lbm_create(nx, ny, ctypes.byref(eos or L.make_eos(0.6)),
                      ctypes.byref(force or L.make_force("GUO")),
                      ctypes.byref(coll or L.make_collision("BGK")), tau, ctypes.byref(h))
    return rc, h


def test_create_validates(L):
    assert _create(L, tau=0.5)[0] == L.LBM_EINVAL
    assert _create(L, nx=0)[0] == L.LBM_EINVAL
    assert _create(L, force=L.make_force("GUO", G=1.0))[0] == L.LBM_EINVAL
    assert _create(L, force=L.make_force("EDM"), coll=L.make_collision("MRT"))[0] == L.LBM_EINVAL
    assert _create(L, coll=L.make_collision("MRT", s=(1.0, 2.5, 1.1, 1.0, 1.1)))[0] == L.LBM_EINVAL
    assert _create(L, eos=L.make_eos(0.6, K=0.0))[0] == L.LBM_EINVAL
    rc, h = _create(L, nx=3, ny=5)
    assert rc == L.LBM_OK and h
    pitch, plane, fb, pb = (ctypes.c_size_t() for _ in range(4))
    assert L.lbm_layout(h, *(ctypes.byref(v) for v in (pitch, plane, fb, pb))) == 0
    assert pitch.value == 64 and plane.value == 64 * 5 and fb.value == 9 * 64 * 5 * 4
    assert L.lbm_set_tile(h, 48, 4) == L.LBM_EINVAL and L.lbm_set_tile(h, 128, 8) == 0
    assert L.lbm_set_probes(h, 3, 0, 0, 0) == L.LBM_EINVAL
    assert L.lbm_set_precision(h, 7) == L.LBM_EINVAL
    # FP32 arithmetic throughout (the value 0) misses the 1e-5 bar and is not offered
    assert L.lbm_set_precision(h, 0) == L.LBM_EINVAL and b"1e-5" in L.lbm_last_error(h)
    assert L.lbm_set_precision(h, L.LBM_PREC_F64) == 0 and L.lbm_set_precision(h, L.LBM_PREC_MIXED) == 0
    # stepping before init is an ordering error, reported without touching the GPU
    assert L.lbm_step(h, 1) == L.LBM_ESTATE
    assert b"init" in L.lbm_last_error(h)
    L.lbm_destroy(h)
    assert L.lbm_strerror(L.LBM_EUNSTABLE) == b"unstable state"


def test_binding_has_no_cpu_path():
    """The product path has no CPU fallback: the binding module only loads the HIP library."""
    src = open(os.path.join(ROOT, "paper_1412_5170_amd", "lbm.py")).read()
    assert "oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_1412_5170_amd")):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_1412_5170_amd", f)).read()


# ---- flat-interface coexistence (host) ---------------------------------------------------

@pytest.mark.parametrize("ttc,K,eps", [(0.6, 1.0, 1.68), (0.6, 0.1, 2.0), (0.8, 1.0, 0.52)])
def test_coexistence_mechanical_matches_oracle(thermo, ttc, K, eps):
    from paper_1412_5170_amd import lbm
    g, l = lbm.coexistence(lbm.make_eos(ttc, K=K), lbm.make_force("GUO"), "mechanical", eps)
    og, ol, _ = thermo.mechanical(ttc, eps, K=K)
    assert g == pytest.approx(og, rel=1e-11) and l == pytest.approx(ol, rel=1e-11)


def test_coexistence_maxwell_matches_oracle(thermo):
    from paper_1412_5170_amd import lbm
    for ttc in (0.5, 0.7, 0.9):
        g, l = lbm.coexistence(lbm.make_eos(ttc), lbm.make_force("GUO"), "maxwell")
        og, ol, _ = thermo.maxwell(ttc)
        assert g == pytest.approx(og, rel=1e-11) and l == pytest.approx(ol, rel=1e-11)


@pytest.mark.parametrize("eps,G", [(1.0, -3.0), (0.0, -4.0)])
def test_coexistence_eq33_consistent(thermo, eps, G):
    """Eq. 33: the mechanical condition with the matching exponent is the Maxwell rule."""
    from paper_1412_5170_amd import lbm
    f = lbm.make_force("GUO", G=G)
    a = lbm.coexistence(lbm.make_ss_eos(eps), f, "maxwell")
    b = lbm.coexistence(lbm.make_ss_eos(eps), f, "mechanical", eps)
    o = thermo.ss_maxwell(eps, G)
    assert a[0] == pytest.approx(o[0], rel=1e-11) and a[1] == pytest.approx(o[1], rel=1e-11)
    assert b[0] == pytest.approx(a[0], rel=1e-11) and b[1] == pytest.approx(a[1], rel=1e-11)


def test_coexistence_rejects_single_phase():
    from paper_1412_5170_amd import lbm
    with pytest.raises(lbm.LBMError):
        lbm.coexistence(lbm.make_ss_eos(1.0), lbm.make_force("GUO", G=-1.0), "maxwell")
    with pytest.raises(lbm.LBMError):
        lbm.coexistence(lbm.make_eos(1.2), lbm.make_force("GUO"), "maxwell")
    with pytest.raises(lbm.LBMError):  # the C-S Maxwell helper does not take Eq. 33
        lbm.eos_maxwell(lbm.make_ss_eos(1.0))


def test_create_accepts_sc_and_eq33_and_rejects_sc_mrt():
    from paper_1412_5170_amd import lbm
    ok = lbm.lbm_create
    import ctypes
    h = lbm._P()
    eos, coll = lbm.make_eos(0.7), lbm.make_collision("BGK")
    assert ok(8, 8, ctypes.byref(eos), ctypes.byref(lbm.make_force("SC")), ctypes.byref(coll),
              1.0, ctypes.byref(h)) == lbm.LBM_OK
    lbm.lbm_destroy(h)
    ss = lbm.make_ss_eos(1.0)
    assert ok(8, 8, ctypes.byref(ss), ctypes.byref(lbm.make_force("GUO", G=-3.0)),
              ctypes.byref(coll), 1.0, ctypes.byref(h)) == lbm.LBM_OK
    lbm.lbm_destroy(h)
    mrt = lbm.make_collision("MRT")
    assert ok(8, 8, ctypes.byref(eos), ctypes.byref(lbm.make_force("SC")), ctypes.byref(mrt),
              1.0, ctypes.byref(h)) == lbm.LBM_EINVAL
    bad = lbm.make_ss_eos(-1.0)
    assert ok(8, 8, ctypes.byref(bad), ctypes.byref(lbm.make_force("GUO", G=-3.0)),
              ctypes.byref(coll), 1.0, ctypes.byref(h)) == lbm.LBM_EINVAL


def test_load_rejects_missing_and_foreign_files(tmp_path):
    from paper_1412_5170_amd import lbm
    h = lbm._P()
    eos, frc, coll = lbm.make_eos(0.7), lbm.make_force("GUO"), lbm.make_collision("BGK")
    assert lbm.lbm_create(8, 8, ctypes.byref(eos), ctypes.byref(frc), ctypes.byref(coll), 1.0,
                          ctypes.byref(h)) == lbm.LBM_OK
    try:
        assert lbm.lbm_load(h, os.fsencode(str(tmp_path / "missing.ckpt"))) == lbm.LBM_EINVAL
        bad = tmp_path / "bad.ckpt"
        bad.write_bytes(b"NOTACKPT" + bytes(64))
        assert lbm.lbm_load(h, os.fsencode(str(bad))) == lbm.LBM_EINVAL
    finally:
        lbm.lbm_destroy(h)


def test_launch_rules_beyond_4gib():
    """Host-side launch rules (no GPU call is made): a lattice above 4 GiB per population
    buffer keeps the sweeps in the rows layout (per-row buffer resources); switching it to the
    planes layout moves it to the two-pass step, and both sweeps are then refused.  The
    default on every lattice is the two-step sweep with 256 threads in XCD order: 16-row segments where that
    gives at least 8192 waves (beyond 4 GiB too, in the rows layout), else 24 rows where that
    gives about 3072, else the height (6 to 24 rows) that gives about 3200 waves, and on small
    lattices fewer rows with one wave per workgroup."""
    from paper_1412_5170_amd import lbm
    eos, frc, coll = lbm.make_eos(0.5, K=1 / 49), lbm.make_force("GUO_LI", sigma=0.125), \
        lbm.make_collision("MRT")

    def create(nx, ny):
        h = lbm._P()
        assert lbm.lbm_create(nx, ny, ctypes.byref(eos), ctypes.byref(frc), ctypes.byref(coll),
                              1.0, ctypes.byref(h)) == lbm.LBM_OK
        return h

    def launch(h):
        v = [ctypes.c_int() for _ in range(4)]
        assert lbm.lbm_get_launch(h, *[ctypes.byref(x) for x in v]) == lbm.LBM_OK
        return tuple(x.value for x in v)

    big = create(10944, 10944)  # 9 x 4 x 10944^2 B = 4.31 GB per buffer
    fb = ctypes.c_size_t()
    assert lbm.lbm_layout(big, None, None, ctypes.byref(fb), None) == lbm.LBM_OK
    assert fb.value > 2 ** 32
    assert launch(big) == (lbm.LBM_KERNEL_SWEEP2, 256, 16, lbm.LBM_LAUNCH_XCD_ORDER)
    assert lbm.lbm_set_launch(big, lbm.LBM_KERNEL_SWEEP, 256, 16, 0) == lbm.LBM_OK
    assert lbm.lbm_set_layout(big, lbm.LBM_LAYOUT_PLANES) == lbm.LBM_OK
    assert launch(big)[0] == lbm.LBM_KERNEL_TWO_PASS
    assert lbm.lbm_set_launch(big, lbm.LBM_KERNEL_SWEEP, 512, 8, 0) == lbm.LBM_EINVAL
    assert lbm.lbm_set_launch(big, lbm.LBM_KERNEL_SWEEP2, 256, 24, 0) == lbm.LBM_EINVAL
    assert lbm.lbm_set_layout(big, lbm.LBM_LAYOUT_ROWS) == lbm.LBM_OK
    assert lbm.lbm_set_launch(big, lbm.LBM_KERNEL_SWEEP, 512, 8, 0) == lbm.LBM_OK
    assert lbm.lbm_set_launch(big, lbm.LBM_KERNEL_SWEEP2, 256, 24, 0) == lbm.LBM_OK
    lbm.lbm_destroy(big)
    small = create(4096, 4096)
    assert launch(small) == (lbm.LBM_KERNEL_SWEEP2, 256, 16, lbm.LBM_LAUNCH_XCD_ORDER)
    assert lbm.lbm_set_layout(small, lbm.LBM_LAYOUT_PLANES) == lbm.LBM_OK
    assert launch(small) == (lbm.LBM_KERNEL_SWEEP2, 256, 16, lbm.LBM_LAUNCH_XCD_ORDER)
    lbm.lbm_destroy(small)
    for n, ty in ((3000, 16), (2048, 24)):  # 52 x 188 = 9776 waves of 16 rows; 36 x 86 = 3096 of 24
        h = create(n, n)
        assert launch(h) == (lbm.LBM_KERNEL_SWEEP2, 256, ty, lbm.LBM_LAUNCH_XCD_ORDER)
        lbm.lbm_destroy(h)
    # smaller lattices: the segment height that gives about 3200 waves, between 6 and 24 rows;
    # where that is 6 rows, 1-12 rows by waves per SIMD and rows per wave, one wave per workgroup
    for n, tx, ty in ((1536, 256, 14), (1152, 256, 8), (1024, 64, 10), (832, 64, 7),
                      (768, 64, 6), (640, 64, 4), (512, 64, 5), (256, 64, 2), (128, 64, 1)):
        h = create(n, n)
        assert launch(h) == (lbm.LBM_KERNEL_SWEEP2, tx, ty, lbm.LBM_LAUNCH_XCD_ORDER)
        lbm.lbm_destroy(h)
    tiny = create(300, 130)  # 6 strips x 130 rows: one row per wave
    assert launch(tiny) == (lbm.LBM_KERNEL_SWEEP2, 64, 1, lbm.LBM_LAUNCH_XCD_ORDER)
    assert lbm.lbm_set_launch(tiny, lbm.LBM_KERNEL_SWEEP2, 320, 32, 0) == lbm.LBM_EINVAL
    assert lbm.lbm_set_launch(tiny, lbm.LBM_KERNEL_SWEEP2, 256, 24, 0) == lbm.LBM_OK
    lbm.lbm_destroy(tiny)


def test_default_two_step_heights_follow_the_wave_count():
    """The default segment height of the two-step sweep, on many lattice shapes (host rule, no
    GPU call): 16 rows where that makes at least 8192 waves of 58 columns, else 24 rows where
    that makes at least 3072, else the lowest height from 6 to 24 rows that keeps the wave count
    at or below about 3200 (one resident round); where that is 6 rows, the height in 1..12 that
    minimises (rows + 4) max(1.5, ceil(waves / 1024)), one wave per workgroup."""
    from paper_1412_5170_amd import lbm
    eos, frc, coll = lbm.make_eos(0.6, K=1 / 49), lbm.make_force("GUO_LI", sigma=0.125), \
        lbm.make_collision("BGK")
    rng = np.random.default_rng(7)
    shapes = [(1, 1), (3, 3), (4, 256), (58, 58), (59, 7), (4096, 8), (8, 4096), (100000, 4),
              (128, 128), (256, 256), (384, 384), (512, 512), (640, 640), (768, 768),
              (832, 832), (1024, 1024), (1152, 1152), (1536, 1536)]
    shapes += [tuple(int(v) for v in rng.integers(1, 6000, 2)) for _ in range(40)]
    for nx, ny in shapes:
        h = lbm._P()
        assert lbm.lbm_create(nx, ny, ctypes.byref(eos), ctypes.byref(frc), ctypes.byref(coll),
                              0.9, ctypes.byref(h)) == lbm.LBM_OK
        v = [ctypes.c_int() for _ in range(4)]
        assert lbm.lbm_get_launch(h, *[ctypes.byref(x) for x in v]) == lbm.LBM_OK
        k, tx, ty, fl = (x.value for x in v)
        lbm.lbm_destroy(h)
        strips = -(-nx // 58)
        waves = lambda rows: strips * -(-ny // rows)  # noqa: E731
        assert (k, fl) == (lbm.LBM_KERNEL_SWEEP2, lbm.LBM_LAUNCH_XCD_ORDER), (nx, ny)
        if waves(16) >= 8192:
            assert (tx, ty) == (256, 16), (nx, ny, ty)
        elif waves(24) >= 3072:
            assert (tx, ty) == (256, 24), (nx, ny, ty)
        elif waves(6) <= 3200:
            cost = {r: (r + 4) * max(1.5, -(-waves(r) // 1024)) for r in range(1, 13)}
            assert tx == 64 and cost[ty] == min(cost.values()), (nx, ny, ty)
            assert all(cost[r] > cost[ty] for r in range(ty + 1, 13)), (nx, ny, ty)
        else:
            assert tx == 256 and 6 < ty <= 24, (nx, ny, ty)
            assert waves(ty) <= 3200 and waves(ty - 1) > 3200, (nx, ny, ty)
