"""ZOOPS and TCM EM on the GPU (em_refine_model, vector path) against the
oracle: J and LLR of every iteration, theta, the final mixing parameter and
the sites, in FP64 (1e-12 relative) and FP32 (1e-5 relative, the tolerance
derived for the FP32-class paths); and the PM_OOPS model equal to em_refine."""
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


def _models(rng, seqs, A, l, k, s, m, beta):
    """theta0 of the instance's enriched buckets (oracle selection)."""
    ref = oracle.Seqs(A, seqs)
    masks = projection_masks(rng, l, k, m)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    bk, mem, _, _ = oracle.select(ref, l, k, RK, RN, s)
    prof = oracle.profile(ref, l, bk, mem)
    bg = oracle.bg_vector(A, None, ref)
    th0 = oracle.theta0(prof, bg, beta)
    return ref, th0, bg


CASES = [
    # name, alphabet, seqs builder, l, k, s, m, iters, beta
    ("dna planted", 4, lambda r: planted_instance(r, 12, 300, 12, 2).seqs, 12, 7, 3, 12, 5, 1.0),
    ("dna ragged half empty", 4,
     lambda r: planted_instance(r, 6, [200, 90, 310, 150, 47, 260], 11, 2).seqs
     + random_sequences(r, 5, [120, 33, 280, 64, 199], "dna"), 11, 6, 3, 10, 4, 0.5),
    ("protein", 20, lambda r: planted_instance(r, 8, 160, 9, 2, alphabet="protein").seqs, 9, 3, 2, 6, 3, 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("model,mix0", [(pm.PM_ZOOPS, 0.5), (pm.PM_ZOOPS, 1.0), (pm.PM_TCM, 0.01),
                                        (pm.PM_TCM, 0.3)],
                         ids=["zoops 0.5", "zoops 1", "tcm 0.01", "tcm 0.3"])
@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_FP32], ids=["fp64", "fp32"])
def test_model_em_matches_oracle(case, model, mix0, prec):
    name, A, make, l, k, s, m, iters, beta = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = make(rng)
    ref, th0, bg = _models(rng, seqs, A, l, k, s, m, beta)
    B = th0.shape[0]
    assert B > 0
    say(f"model em {name} model={model} mix0={mix0} prec={prec} B={B}")
    r_th, r_mix, r_J, r_LL, r_sites = oracle.em_model(ref, l, model, mix0, th0, bg, iters, beta)
    S = pm.Seqs(A, seqs)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    th = torch.zeros((B, A, l), dtype=torch.float64, device="cuda")
    mix = torch.zeros(B, dtype=torch.float64, device="cuda")
    J = torch.zeros((B, iters + 1), dtype=torch.float64, device="cuda")
    LL = torch.zeros_like(J)
    sites = torch.zeros((B, len(seqs)), dtype=torch.int32, device="cuda")
    pm.em_refine_model(S, l, model, mix0, d(th0), d(bg), B, None, iters, beta, prec, th, mix, J, LL, sites)
    torch.cuda.synchronize()
    rtol = 1e-12 if prec == pm.PM_FP64 else 1e-5
    scale = np.abs(r_J).max()
    np.testing.assert_allclose(J.cpu().numpy(), r_J, rtol=rtol, atol=rtol * scale)
    np.testing.assert_allclose(LL.cpu().numpy(), r_LL, rtol=rtol, atol=rtol * scale)
    np.testing.assert_allclose(th.cpu().numpy(), r_th, rtol=2 * rtol, atol=2 * rtol)
    np.testing.assert_allclose(mix.cpu().numpy(), r_mix, rtol=2 * rtol, atol=1e-15)
    got = sites.cpu().numpy()
    if prec == pm.PM_FP64:
        assert np.array_equal(got, r_sites)
    else:
        # FP32 scores: a site may differ only where the oracle's decision is
        # within rounding (near-tied best starts or a site mass near 1/2)
        assert np.mean(got == r_sites) > 0.97


def test_oops_model_is_em_refine():
    rng = np.random.default_rng(3)
    seqs = planted_instance(rng, 10, 200, 10, 2).seqs
    ref, th0, bg = _models(rng, seqs, 4, 10, 6, 3, 8, 1.0)
    B = th0.shape[0]
    S = pm.Seqs(4, seqs)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    outs = []
    for use_model in (True, False):
        th = torch.zeros((B, 4, 10), dtype=torch.float64, device="cuda")
        J = torch.zeros((B, 4), dtype=torch.float64, device="cuda")
        if use_model:
            pm.em_refine_model(S, 10, pm.PM_OOPS, 0.0, d(th0), d(bg), B, None, 3, 1.0, pm.PM_FP64, th, None, J)
        else:
            pm.em_refine(S, 10, d(th0), d(bg), B, None, 3, 1.0, pm.PM_FP64, th, J)
        torch.cuda.synchronize()
        outs.append((th.cpu().numpy(), J.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_model_em_rejects_bad_arguments():
    rng = np.random.default_rng(4)
    seqs = random_sequences(rng, 3, 40, "dna")
    S = pm.Seqs(4, seqs)
    th0 = torch.full((1, 4, 8), 0.25, dtype=torch.float64, device="cuda")
    bg = torch.full((4,), 0.25, dtype=torch.float64, device="cuda")
    th = torch.zeros_like(th0)
    J = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    for model, mix, prec in ((pm.PM_ZOOPS, 0.0, pm.PM_FP64), (pm.PM_TCM, 1.5, pm.PM_FP64),
                             (pm.PM_ZOOPS, 0.5, pm.PM_F16X2), (7, 0.5, pm.PM_FP64)):
        with pytest.raises(pm.PmError) as e:
            pm.em_refine_model(S, 8, model, mix, th0, bg, 1, None, 1, 1.0, prec, th, None, J)
        assert e.value.code == pm.PM_EINVAL
