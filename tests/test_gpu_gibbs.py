"""Gibbs site sampling (gibbs_refine) on the GPU against the oracle's
sampler: the same Philox4x64-10 draws give the same chains, so the best
alignment's sites are equal, and F of every sweep and the answer's theta
agree to FP64 rounding (1e-12 relative); the chains of different models and
seeds differ; bad arguments are refused."""
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from synth import planted_instance, projection_masks, random_sequences

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def _bucket_models(rng, seqs, A, l, k, s, m, beta, cap=None):
    ref = oracle.Seqs(A, seqs)
    masks = projection_masks(rng, l, k, m)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    bk, mem, _, _ = oracle.select(ref, l, k, RK, RN, s)
    prof = oracle.profile(ref, l, bk, mem)
    bg = oracle.bg_vector(A, None, ref)
    th0 = oracle.theta0(prof, bg, beta)
    return ref, (th0 if cap is None else th0[:cap]), bg


CASES = [
    # name, alphabet, seqs builder, l, k, s, m, sweeps, beta, seed
    ("dna planted", 4, lambda r: planted_instance(r, 12, 300, 12, 2).seqs, 12, 7, 3, 10, 8, 1.0, 5),
    ("dna ragged long", 4, lambda r: planted_instance(r, 9, [150, 2100, 64, 777, 300, 1500, 90, 1024, 33],
                                                      11, 2).seqs, 11, 6, 3, 6, 5, 0.5, 77),
    ("protein", 20, lambda r: planted_instance(r, 8, 200, 10, 2, alphabet="protein").seqs, 10, 3, 2, 5, 6, 1.0,
     123456789),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_gibbs_matches_oracle(case):
    name, A, make, l, k, s, m, sweeps, beta, seed = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = make(rng)
    ref, th0, bg = _bucket_models(rng, seqs, A, l, k, s, m, beta, cap=300)
    B = th0.shape[0]
    assert B > 8
    say(f"gibbs {name} B={B}")
    r_th, r_F, r_sites = oracle.gibbs(ref, l, th0, bg, sweeps, beta, seed)
    S = pm.Seqs(A, seqs)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    th = torch.zeros((B, A, l), dtype=torch.float64, device="cuda")
    F = torch.zeros((B, sweeps + 1), dtype=torch.float64, device="cuda")
    sites = torch.zeros((B, len(seqs)), dtype=torch.int32, device="cuda")
    pm.gibbs_refine(S, l, d(th0), d(bg), B, None, sweeps, beta, seed, th, F, sites)
    torch.cuda.synchronize()
    assert np.array_equal(sites.cpu().numpy(), r_sites)
    np.testing.assert_allclose(F.cpu().numpy(), r_F, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(th.cpu().numpy(), r_th, rtol=1e-12, atol=1e-15)


def test_gibbs_respects_the_device_count_and_the_seed():
    rng = np.random.default_rng(8)
    seqs = planted_instance(rng, 10, 250, 10, 2).seqs
    ref, th0, bg = _bucket_models(rng, seqs, 4, 10, 6, 3, 8, 1.0, cap=64)
    B = th0.shape[0]
    S = pm.Seqs(4, seqs)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    th = torch.full((B, 4, 10), -1.0, dtype=torch.float64, device="cuda")
    F = torch.zeros((B, 6), dtype=torch.float64, device="cuda")
    n_dev = torch.tensor([B - 5], dtype=torch.int64, device="cuda")
    say("gibbs n_dev")
    pm.gibbs_refine(S, 10, d(th0), d(bg), B, n_dev, 5, 1.0, 3, th, F)
    torch.cuda.synchronize()
    got = th.cpu().numpy()
    assert np.all(got[B - 5:] == -1.0) and np.all(got[:B - 5] > 0)
    r_th, r_F, _ = oracle.gibbs(ref, 10, th0[:B - 5], bg, 5, 1.0, 3)
    np.testing.assert_allclose(F.cpu().numpy()[:B - 5], r_F, rtol=1e-12)
    F2 = torch.zeros_like(F)
    pm.gibbs_refine(S, 10, d(th0), d(bg), B, None, 5, 1.0, 4, torch.zeros_like(th), F2)
    torch.cuda.synchronize()
    assert not np.array_equal(F2.cpu().numpy()[:, 1:], F.cpu().numpy()[:, 1:])


def test_gibbs_rejects_bad_arguments():
    rng = np.random.default_rng(9)
    S = pm.Seqs(4, random_sequences(rng, 3, 40, "dna"))
    th0 = torch.full((1, 4, 8), 0.25, dtype=torch.float64, device="cuda")
    bg = torch.full((4,), 0.25, dtype=torch.float64, device="cuda")
    th = torch.zeros_like(th0)
    for beta, sweeps in ((0.0, 2), (1.0, -1)):
        with pytest.raises(pm.PmError) as e:
            pm.gibbs_refine(S, 8, th0, bg, 1, None, sweeps, beta, 1, th)
        assert e.value.code == pm.PM_EINVAL
