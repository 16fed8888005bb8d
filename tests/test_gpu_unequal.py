"""GPU parity of unequal splits (emu_dgemm_ab: B with fewer slices than A,
t = s + 1) against the oracle's dgemm_emu(..., s_b=...) bit for bit, and the
product-count reduction that changes no bit: B whose columns carry only
s_b digits gives the same result as the full count."""
import ctypes

import numpy as np
import pytest
import torch

import matgen
import oracle as O
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _same_bits(a, b):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("m,n,k,s,sb", [(200, 300, 500, 9, 2), (130, 257, 700, 9, 8),
                                        (300, 90, 333, 5, 1), (64, 64, 64, 3, 2),
                                        (257, 255, 1000, 7, 4), (512, 512, 14000, 9, 6)])
def test_unequal_splits_bit_exact(m, n, k, s, sb):
    A = matgen.phi_matrix(m, k, 2.0, seed=61, substream=0)
    B = matgen.phi_matrix(k, n, 1.0, seed=61, substream=1)
    C0 = matgen.uniform(m, n, seed=61, substream=2)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
        Cg = emu.colmajor(C0)
        emu.dgemm(Ag, Bg, Cg, alpha=alpha, beta=beta, nslices=s, nslices_b=sb)
        ref = O.dgemm_emu(A, B, s, alpha=alpha, beta=beta, C=C0, s_b=sb)
        assert _same_bits(_host(Cg), ref), (alpha, beta)


def test_fewer_slices_for_a_two_digit_operand_change_no_bit():
    m, n, k = 384, 256, 2048
    g = np.random.default_rng(62)
    B = g.integers(-(2 ** 14) + 1, 2 ** 14, size=(k, n)).astype(np.float64)
    B[0, :] = 2.0 ** 14 - 1
    B = np.asfortranarray(B)
    A = matgen.phi_matrix(m, k, 1.0, seed=62)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    full = _host(emu.dgemm(Ag, Bg, nslices=9))
    two = _host(emu.dgemm(Ag, Bg, nslices=9, nslices_b=2))
    assert _same_bits(full, two)
    assert _same_bits(two, O.dgemm_emu(A, B, 9, s_b=2))


def test_unequal_splits_refuse_k_beyond_one_pass():
    # eight pairs per diagonal fit one exact INT32 pass up to k = 16640:
    # k = 17000 with s_b = 8 is refused before any launch, while s_b = s
    # (the plain method) takes its chunked path
    k = 17000
    A = torch.zeros((k, 16), dtype=torch.float64, device="cuda").t()     # 16 x k, ld 16
    B = torch.zeros((16, k), dtype=torch.float64, device="cuda").t()     # k x 16, ld k
    C = torch.zeros((16, 16), dtype=torch.float64, device="cuda").t()
    args = (16, 16, k, ctypes.c_double(1.0), A.data_ptr(), 16, B.data_ptr(), k,
            ctypes.c_double(0.0), C.data_ptr(), 16)
    assert emu.emu_dgemm_ab(*args, 9, 8) == emu.EMU_ERR_UNSUPPORTED
    assert "one-pass" in emu.emu_last_error()
    assert emu.emu_dgemm_ab(*args, 9, 9) == 0
    torch.cuda.synchronize()
    assert bool((C == 0).all())
