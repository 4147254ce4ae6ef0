"""The C-ABI library loads, exports what include/mot_jvie.h declares, and its
host-side integer helpers agree bit-exactly with the oracle (no GPU needed)."""

import ctypes
import os
import re

import pytest

from oracle import basis, masks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mot_jvie.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("build_green_spectra", "z0_matvec", "history_update", "mot_step", "mot_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_28309_amd import native
    lib = ctypes.CDLL(native.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(native.EXPORTS) == set(_declared())


def test_binding_uses_torchs_hip_runtime():
    # importing the binding first must not map a second HIP runtime beside
    # torch's (torch's device memory and streams belong to its own copy)
    import subprocess
    import sys
    code = ("import paper_2607_28309_amd.native, torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1 and os.path.dirname(libs[0]).endswith(os.path.join("torch", "lib")), libs


@pytest.mark.parametrize("n,alpha", [((16, 16, 16), 1), ((64, 64, 64), 8), ((96, 96, 96), 1),
                                     ((320, 320, 48), 16), ((9, 7, 5), 3), ((1, 1, 1), 4)])
def test_nlags_bit_exact(n, alpha):
    from paper_2607_28309_amd import native
    assert native.nlags(*n, alpha=alpha) == basis.nlags(*n, alpha=alpha)
    assert native.nlags(*n, cdt=0.7) == basis.nlags(*n, cdt=0.7)


@pytest.mark.parametrize("n,k,alpha,cdt", [((12, 10, 8), 0, 1, 0.0), ((12, 10, 8), 3, 2, 0.0),
                                           ((7, 9, 5), 5, 3, 0.0), ((10, 6, 4), 0, 0, 1.1992),
                                           ((10, 6, 4), 4, 0, 0.83)])
def test_zk_nnz_bit_exact(n, k, alpha, cdt):
    from paper_2607_28309_amd import native
    ref = masks.zk_nnz(*n, k=k, alpha=alpha if alpha else None, cdt=cdt if not alpha else None)
    assert native.zk_nnz(*n, k=k, alpha=alpha, cdt=cdt) == ref


@pytest.mark.parametrize("alpha", [1, 2, 4, 8, 16])
def test_z0_nnz_nested_cube_sweep(alpha):
    """Z0 nonzeros of the 96^3 time-step sweep, library against the oracle's
    mask count (the growth of the causal region with the time step)."""
    from paper_2607_28309_amd import native
    assert native.zk_nnz(96, 96, 96, k=0, alpha=alpha) == masks.zk_nnz(96, 96, 96, k=0, alpha=alpha)


def test_table3_rows_from_library():
    # Table III (Sec. III-B): 40^3/alpha=4 -> 9.24e6 and 80^3/alpha=2 -> 76.09e6
    from paper_2607_28309_amd import native
    c0 = 299.792458
    assert native.zk_nnz(40, 40, 40, 0, cdt=4 * 0.005 * c0 / 5.0) == 9236568
    assert native.zk_nnz(80, 80, 80, 0, cdt=2 * 0.005 * c0 / 2.5) == 76092408


def test_lengths_and_invalid_grids():
    from paper_2607_28309_amd import native
    for n in (16, 32, 96, 128, 640):
        assert native.length_supported(n)
    for n in (7, 14, 1000):
        assert not native.length_supported(n)
    h = ctypes.c_void_p()
    for g in (native.make_grid(15, 8, 8, 1), native.make_grid(16, 8, 8, -1), native.make_grid(16, 7, 8, 1),
              native.make_grid(0, 8, 8, 1), native.make_grid(16, 8, 8, 0, 0.0)):
        assert native.LIB.mot_create(ctypes.byref(g), 0, None, ctypes.byref(h)) == native.MOT_EINVAL
    assert native.LIB.mot_create(ctypes.byref(native.make_grid(16, 8, 8, 1)), 7, None, ctypes.byref(h)) == \
        native.MOT_EINVAL
    assert native.LIB.mot_strerror(native.MOT_ENOCONV) == b"TFQMR did not converge"


def test_setters_reject_a_null_context():
    # argument checks before any device work: a NULL context is MOT_EINVAL
    from paper_2607_28309_amd import native
    assert native.LIB.mot_set_wide_offsets(None, 0) == native.MOT_EINVAL
    assert native.LIB.mot_set_history_scheme(None, 1) == native.MOT_EINVAL
    assert native.LIB.mot_set_graphs(None, 0) == native.MOT_EINVAL
