"""emu_dgemm_noalloc (scratch in the library's fixed device array, no
allocation) against emu_dgemm on the same inputs, bit for bit: a long-K
product that takes the chunked path, then a smaller one, then a shape too
large for the fixed array (rejected before any launch)."""
import ctypes

import numpy as np
import pytest
import torch

import matgen
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _run(fn, A, B, C0, alpha, beta, s):
    Ag, Bg, Cg = emu.colmajor(A), emu.colmajor(B), emu.colmajor(C0)
    m, k = A.shape
    n = B.shape[1]
    rc = fn(m, n, k, ctypes.c_double(alpha), Ag.data_ptr(), Ag.stride(1), Bg.data_ptr(),
            Bg.stride(1), ctypes.c_double(beta), Cg.data_ptr(), Cg.stride(1), s)
    return rc, Cg


def test_noalloc_matches_dgemm_on_two_calls_and_rejects_oversize():
    torch.cuda.set_device(0)
    cases = [(64, 96, 20000, 9, 3.0, -0.5, 1.25), (200, 150, 300, 7, 2.0, 1.0, 0.0)]
    for i, (m, n, k, s, phi, alpha, beta) in enumerate(cases):
        A = matgen.phi_matrix(m, k, phi, seed=90 + i, substream=0)
        B = matgen.phi_matrix(k, n, phi, seed=90 + i, substream=1)
        C0 = matgen.uniform(m, n, seed=90 + i, substream=2)
        need = emu.emu_workspace_bytes(m, n, k, s)
        assert 0 < need <= emu.EMU_NOALLOC_SCRATCH_BYTES
        rc_ref, Cref = _run(emu.emu_dgemm, A, B, C0, alpha, beta, s)
        assert rc_ref == 0
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        rc, Cg = _run(emu.emu_dgemm_noalloc, A, B, C0, alpha, beta, s)
        assert rc == 0, emu.emu_last_error()
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        got, ref = Cg.cpu().numpy(), Cref.cpu().numpy()
        assert np.array_equal(got.view(np.int64), ref.view(np.int64)), (m, n, k, s)
        # the call itself took no device memory (Cg was allocated before free0)
        assert free1 == free0
    # a shape whose scratch exceeds the fixed array: EMU_ERR_WORKSPACE, C untouched
    m = n = k = 4096
    assert emu.emu_workspace_bytes(m, n, k, 9) > emu.EMU_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((k, m), dtype=torch.float64, device="cuda").t()
    B = torch.zeros((n, k), dtype=torch.float64, device="cuda").t()
    C = torch.full((n, m), 7.0, dtype=torch.float64, device="cuda").t()
    rc = emu.emu_dgemm_noalloc(m, n, k, ctypes.c_double(1.0), A.data_ptr(), m, B.data_ptr(), k,
                               ctypes.c_double(0.0), C.data_ptr(), m, 9)
    assert rc == emu.EMU_ERR_WORKSPACE
    assert "fixed" in emu.emu_last_error()
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())
