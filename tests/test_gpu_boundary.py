"""GPU checks of the boundary's scratch rules: a caller-registered workspace,
threads calling concurrently on their own streams, and one thread moving
between streams (every result compared with the oracle bit for bit)."""
import threading

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


def test_registered_workspace_gives_the_same_bits_and_too_small_fails():
    m, n, k, s = 300, 200, 500, 7
    A = matgen.phi_matrix(m, k, 2.0, seed=81, substream=0)
    B = matgen.phi_matrix(k, n, 2.0, seed=81, substream=1)
    ref = O.dgemm_emu(A, B, s)
    need = emu.emu_workspace_bytes(m, n, k, s)
    assert need > 0
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    try:
        emu.set_workspace(buf)
        Cg = emu.dgemm(emu.colmajor(A), emu.colmajor(B), nslices=s)
        torch.cuda.synchronize()
        assert _same_bits(Cg.cpu().numpy(), ref)
        # LU in a workspace of exactly the size the query names
        M = matgen.phi_matrix(700, 700, 1.0, seed=82)
        wl = torch.empty(emu.emu_getrf_workspace_bytes(700, 700, 128, 5), dtype=torch.uint8,
                         device="cuda")
        emu.set_workspace(wl)
        Mg = emu.colmajor(M)
        ipiv, info = emu.dgetrf(Mg, nb=128, nslices=5)
        torch.cuda.synchronize()
        LU, piv, _ = O.getrf(M, nb=128, s=5)
        assert _same_bits(Mg.cpu().numpy(), LU) and np.array_equal(ipiv.cpu().numpy(), piv)
        # one byte short of what the GEMM needs
        emu.set_workspace(buf[:need - 1])
        with pytest.raises(emu.EmuError) as ex:
            emu.dgemm(emu.colmajor(A), emu.colmajor(B), nslices=s)
        assert "1002" in str(ex.value) and str(need) in str(ex.value)
    finally:
        emu.set_workspace(None)


def test_threads_on_their_own_streams():
    shapes = [(257, 190, 300, 5), (130, 400, 77, 9), (512, 64, 1000, 3)]
    cases = []
    for i, (m, n, k, s) in enumerate(shapes):
        A = matgen.phi_matrix(m, k, 3.0, seed=83, substream=2 * i)
        B = matgen.phi_matrix(k, n, 3.0, seed=83, substream=2 * i + 1)
        cases.append((A, B, s, O.dgemm_emu(A, B, s)))
    out = [None] * len(cases)
    errors = []

    def work(i):
        try:
            A, B, s, _ = cases[i]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                Ag, Bg = emu.colmajor(A), emu.colmajor(B)
                res = []
                for _ in range(4):
                    res.append(emu.dgemm(Ag, Bg, nslices=s))
                st.synchronize()
                out[i] = [r.cpu().numpy() for r in res]
        except Exception as e:          # reported in the main thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i, (_, _, _, ref) in enumerate(cases):
        for r in out[i]:
            assert _same_bits(r, ref), i


def test_one_thread_moving_between_streams():
    # a long product on one stream, then a small one on another stream that
    # reuses the same scratch: the second must wait for the first
    A = matgen.phi_matrix(1024, 4096, 1.0, seed=84, substream=0)
    B = matgen.phi_matrix(4096, 1024, 1.0, seed=84, substream=1)
    a = matgen.phi_matrix(100, 50, 1.0, seed=84, substream=2)
    b = matgen.phi_matrix(50, 90, 1.0, seed=84, substream=3)
    Ag, Bg, ag, bg = (emu.colmajor(x) for x in (A, B, a, b))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        C = emu.dgemm(Ag, Bg, nslices=9)
    with torch.cuda.stream(s2):
        c = emu.dgemm(ag, bg, nslices=4)
    torch.cuda.synchronize()
    assert _same_bits(C.cpu().numpy(), O.dgemm_emu(A, B, 9))
    assert _same_bits(c.cpu().numpy(), O.dgemm_emu(a, b, 4))
