"""C-ABI library: loads, exports every declared symbol, host-only logic (no GPU calls)."""
import os
import re

import numpy as np
import pytest

import paper_2402_05283_amd as cp
from paper_2402_05283_amd import _lib
from oracle import cpra as OC
from oracle import stepd as OD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cpra.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cpra_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = cp.load()
    names = _declared()
    assert "cpra_plan" in names and "cpra_plan_create" in names and "cpra_iterate" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTED) == names


def test_workspace_size_and_validation():
    p = cp.make_params(512, 360)
    n = cp.workspace_size(p)
    # P, Pmid (complex64 half spectra), two real iterates, amplitude pairs: >= 5 planes of N*N*4 bytes
    assert n >= 360 * 512 * 512 * 4 * 5
    p16 = cp.make_params(512, 360, amp=cp.AMP_F16)
    assert cp.workspace_size(p16) < n
    p64 = cp.make_params(512, 360, real=cp.REAL_F64)
    assert cp.workspace_size(p64) > n
    bad = [
        dict(N=100, Np=4), dict(N=64, Np=0), dict(N=64, Np=4, n_ei=0), dict(N=64, Np=4, alpha=(0.5, 0.6, 0.2)),
        dict(N=64, Np=4, alpha=(-0.1, 1.0, 0.1)), dict(N=64, Np=4, real=cp.REAL_F64, amp=cp.AMP_F16),
        dict(N=64, Np=4, wrap=7), dict(N=64, Np=4, theta=[0.0, np.nan, 1.0, 2.0]), dict(N=64, Np=4, insertion=2),
        dict(N=64, Np=4, n_guess=-1),
    ]
    for kw in bad:
        with pytest.raises(cp.CpraError) as e:
            cp.workspace_size(cp.make_params(**kw))
        assert e.value.status in (-1, -5)
    with pytest.raises(cp.CpraError) as e:
        cp.workspace_size(cp.make_params(100, 4))
    assert e.value.status == -5 and "N must be" in str(e.value)


@pytest.mark.parametrize("N,Np", [(16, 7), (64, 16), (192, 90), (256, 180), (512, 360)])
def test_slice_cells_bit_exact_vs_oracle(N, Np):
    theta = np.pi * np.arange(Np) / Np
    kx, ky = cp.slice_cells(N, Np)
    okx, oky = OD.slice_cells(N, theta)
    # oracle: centred indices; library: native indices (centred - N/2 mod N)
    assert np.array_equal(kx, (okx - N // 2) % N)
    assert np.array_equal(ky, (oky - N // 2) % N)
    kx2, ky2 = cp.slice_cells(N, Np, theta)
    assert np.array_equal(kx, kx2) and np.array_equal(ky, ky2)


def test_slice_cells_explicit_angles():
    rng = np.random.default_rng(0)
    theta = np.sort(rng.uniform(0, np.pi, 23))
    kx, ky = cp.slice_cells(128, 23, theta)
    okx, oky = OD.slice_cells(128, theta)
    assert np.array_equal(kx, (okx - 64) % 128) and np.array_equal(ky, (oky - 64) % 128)


@pytest.mark.parametrize("wrap", [cp.WRAP_MIRROR, cp.WRAP_PLAIN])
def test_coupling_table_matches_oracle(wrap):
    Np = 9
    alpha = (0.1, 0.6, 0.3)
    rng = np.random.default_rng(1)
    for present in (np.ones(Np, np.uint8), (rng.uniform(size=Np) < 0.6).astype(np.uint8)):
        present[3] = 1
        p = cp.make_params(64, Np, alpha=alpha, wrap=wrap)
        left, right, w, mirror = cp.coupling_table(p, present)
        ref = OC.coupling_weights(Np, present.astype(bool), alpha, wrap)
        for n in range(Np):
            (l, wl, ml), w0, (r, wr, mr) = ref[n]
            assert (left[n], right[n]) == (l, r)
            assert (bool(mirror[n, 0]), bool(mirror[n, 1])) == (ml, mr)
            assert np.allclose(w[n], [wl, w0, wr], rtol=0, atol=1e-15)


def test_single_angle_coupling_table():
    p = cp.make_params(64, 1, alpha=(0.25, 0.5, 0.25))
    left, right, w, mirror = cp.coupling_table(p)
    assert left[0] == 0 and right[0] == 0 and mirror[0].tolist() == [1, 1]


def test_iterate_batch_argument_checks_need_no_device():
    """Argument errors of cpra_iterate_batch are reported before any device call."""
    import ctypes
    lib = cp.load()
    assert lib.cpra_iterate_batch(None, 1, 1, 0, 0.9) == -1
    one_null = (ctypes.c_void_p * 1)(None)
    assert lib.cpra_iterate_batch(one_null, 1, 1, 0, 0.9) == -1
    assert b"NULL" in lib.cpra_last_error(None)
    assert lib.cpra_iterate_batch(one_null, -1, 1, 0, 0.9) == -1
    assert lib.cpra_iterate_batch(one_null, 0, 1, 0, 0.9) == 0      # nothing to do
