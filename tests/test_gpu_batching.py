"""Batching helpers on the GPU: waves of uneven problems and the launch-shape autotuner."""

import json

import numpy as np
import pytest

from workloads import random_sparse_symmetric, simple_cubic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _S():
    import paper_0802_0748_amd as S

    return S


def test_waves_equal_one_batched_solve():
    """greens_diag_waves splits uneven problems into waves that fit a byte budget; each
    right-hand side gets the same bits as in one batched solve (a right-hand side's
    arithmetic does not depend on what it is batched with)."""
    S = _S()
    rng = np.random.default_rng(31)
    Ls = [5, 8, 6, 7, 4]
    Hcs = [simple_cubic(L, rng.uniform(-2, 2, L ** 3)) for L in Ls]
    Hs = [S.Hamiltonian.from_csr(h) for h in Hcs]
    rhs = [np.sort(rng.choice(h.n, size=3, replace=False)) for h in Hcs]
    z = np.linspace(-6, 6, 12) + 0.1j
    G1, rep1, rc1 = S.greens_diag_batched(Hs, z, rhs, tol=1e-10, max_iter=4000)
    budget = 16 * len(z) * 3 * 8 ** 3  # the largest problem alone
    Gw, repw, rcw, waves = S.greens_diag_waves(Hs, z, rhs, max_bytes=budget, tol=1e-10, max_iter=4000)
    assert len(waves) >= 3
    assert sorted(q for w in waves for q in w) == list(range(len(Ls)))
    assert rc1 == rcw == 0
    for q in range(len(Ls)):
        assert np.array_equal(Gw[q].cpu().numpy(), G1[q].cpu().numpy())
        assert np.array_equal(repw[q]["iters"], rep1[q]["iters"])


def test_tuner_returns_a_candidate_and_caches_it(tmp_path):
    """The tuner times each candidate shape on the problem itself, keeps the fastest, and
    answers from its cache the second time; a solve with the tuned shape gives the same
    bits as the default shape in the step form of the update (block length and shifts per
    workgroup change only the schedule of the same arithmetic)."""
    from paper_0802_0748_amd import tune

    S = _S()
    rng = np.random.default_rng(32)
    Hc = random_sparse_symmetric(1500, 0.004, rng, diag_scale=2.0)
    H = S.Hamiltonian.from_csr(Hc)
    z = np.linspace(-3, 3, 40) + 0.05j
    B = torch.from_numpy(rng.normal(size=(4, Hc.n)) + 1j * rng.normal(size=(4, Hc.n))).cuda()
    cache = str(tmp_path / "tune.json")
    best = tune.tune(H, z, B, iters=48, cache=cache, blocks=(8, 24), shifts_per_wg=(16, 32))
    assert best["block"] in (8, 24) and best["shifts_per_wg"] in (16, 32) and best["ms_per_iter"] > 0
    assert len(best["candidates"]) == 4
    with open(cache) as f:
        table = json.load(f)
    assert list(table.values())[0] == best
    again = tune.tune(H, z, B, iters=48, cache=cache, blocks=(8, 24), shifts_per_wg=(16, 32))
    assert again == best
    Xt, rept, _, _ = S.shifted_cocg_solve(H, z, B, tol=1e-10, max_iter=3000, block=best["block"],
                                          shifts_per_wg=best["shifts_per_wg"], update_form="step")
    Xd, repd, _, _ = S.shifted_cocg_solve(H, z, B, tol=1e-10, max_iter=3000, update_form="step")
    assert np.array_equal(rept["iters"], repd["iters"])
    assert np.array_equal(Xt.cpu().numpy(), Xd.cpu().numpy())
