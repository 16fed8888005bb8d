"""GPU checks of the batched precision form (emu_dgesv_batched_ir): every
system of an uneven batch against the oracle's single-system refinement
(gesv_ir at the same block size): same final slice count, iteration counts
within one, double-double backward error <= 1e-15, and solutions within
1e-12 of the oracle's where the system is well conditioned; one
ill-conditioned system (randsvd, kappa 1e10) that must fall back to more
slices; inputs untouched."""
import numpy as np
import pytest
import torch

import matgen
import oracle as O
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("s", [3, 5])
def test_batched_refinement_matches_single_system_oracle(s):
    specs = matgen.batched_specs(14, seed=5, nmax=400)
    As = [matgen.phi_matrix(n, n, phi, seed=5, substream=1000 + i)
          for i, (n, phi, r) in enumerate(specs)]
    Bs = [matgen.uniform(n, r, seed=5, substream=5000 + i) for i, (n, phi, r) in enumerate(specs)]
    # an ill-conditioned member: refinement from few slices cannot converge
    As.append(matgen.kappa_matrix(300, 1.0, 1e10, seed=6, variant="randsvd"))
    Bs.append(matgen.uniform(300, 2, seed=6, substream=1))
    Ag = [emu.colmajor(a) for a in As]
    Bg = [emu.colmajor(b) for b in Bs]
    A0 = [a.clone() for a in Ag]
    Xs, inf = emu.dgesv_batched_ir(Ag, Bg, nb=32, nslices=s, tol=1e-15)
    assert inf["rc"] == 0
    for i, (A, B) in enumerate(zip(As, Bs)):
        Xo, io = O.gesv_ir(A, B, nb=32, s=s, tol=1e-15)
        X = _host(Xs[i])
        assert inf["info"][i] == 0 and io["converged"]
        assert inf["s_final"][i] == io["s_final"], i
        assert abs(inf["iters"][i] - io["iters"]) <= 1, i
        assert O.backward_error(A, X, B) <= 1e-15, i
        assert inf["berr"][i] <= 1e-15
        if i < len(specs):
            assert np.abs(X - Xo).max() <= 1e-12 * np.abs(Xo).max(), i
        assert torch.equal(Ag[i], A0[i])
    if s == 3:
        assert inf["s_final"][-1] > s      # the kappa = 1e10 system fell back


def test_batched_refinement_reports_singular_system():
    A1 = matgen.phi_matrix(100, 100, 1.0, seed=7)
    A2 = np.array(matgen.phi_matrix(150, 150, 1.0, seed=8), order="F")
    A2[:, 40] = 0.0
    Bs = [matgen.uniform(100, 1, seed=9), matgen.uniform(150, 1, seed=10)]
    Xs, inf = emu.dgesv_batched_ir([emu.colmajor(A1), emu.colmajor(A2)],
                                   [emu.colmajor(b) for b in Bs], nb=32, nslices=5)
    assert inf["rc"] == 0
    assert inf["info"] == [0, 41]
    assert O.backward_error(A1, _host(Xs[0]), Bs[0]) <= 1e-15
