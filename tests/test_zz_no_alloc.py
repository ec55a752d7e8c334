"""The allocation-free Newton solve (spsvm_newton_solve_noalloc) against the workspace entry point it varies
(spsvm_newton_solve), through the C ABI: two calls in a row, the second on a smaller system, each bit for bit equal to
the workspace call on the same input (same kernels; the static scratch keeps the previous call's contents)."""

import numpy as np
import pytest
import torch

import paper_1404_1066_amd as lib

pytestmark = pytest.mark.gpu


def _system(m, seed):
    r = np.random.default_rng(seed)
    A = r.standard_normal((m, m + 5))
    H = A @ A.T / (m + 5) + 0.5 * np.eye(m)
    return torch.tensor(H, device="cuda"), torch.tensor(r.standard_normal(m), device="cuda")


def test_noalloc_solve_equals_workspace_solve_twice():
    for m, seed in ((4000, 1), (700, 2)):  # past the one-workgroup solves, then a smaller system in the same scratch
        H, g = _system(m, seed)
        Ha, Hb = H.clone(), H.clone()
        xa = lib.newton_solve(Ha, g)
        xb = lib.newton_solve_noalloc(Hb, g)
        assert torch.equal(xa, xb)
        assert torch.equal(torch.tril(Ha), torch.tril(Hb))
        want = -np.linalg.solve(H.cpu().numpy(), g.cpu().numpy())
        assert np.max(np.abs(xb.cpu().numpy() - want)) <= 1e-11 * np.max(np.abs(want))


def test_noalloc_solve_limits_and_not_pd():
    with pytest.raises(lib.SpsvmError) as e:  # rejected before any GPU work
        lib.newton_solve_noalloc(torch.zeros((4097, 1), dtype=torch.float64, device="cuda"),
                                 torch.zeros(4097, dtype=torch.float64, device="cuda"))
    assert e.value.status == 1 and "4096" in str(e.value)
    H = torch.tensor(np.diag([1.0, -1.0, 2.0]), device="cuda")
    with pytest.raises(lib.SpsvmError) as e:
        lib.newton_solve_noalloc(H, torch.ones(3, dtype=torch.float64, device="cuda"))
    assert e.value.status == 4
    H, g = _system(5, 3)  # the flag left set by the failed call is cleared by the next one
    assert torch.equal(lib.newton_solve_noalloc(H.clone(), g), lib.newton_solve(H.clone(), g))
