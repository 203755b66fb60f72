"""Checkpoint and resume of the dynamic state (csc_dyn_export / csc_dyn_import) through the C
ABI: a resumed sequence is bit-identical to an uninterrupted one, and an edited cut-off in
the exported state forces the refinement of Algorithm 1 step 7 exactly as in the oracle."""

import numpy as np
import pytest
import torch

from oracle import dynamic
from workloads import DynamicSBM, sbm
from helpers import rel_fro, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def seq():
    g0 = sbm(2000, 4, 20.0, 0.05, seed=111)
    dyn = DynamicSBM(g0, seed=112)
    return [g0] + [dyn.step(0.01, 0.005) for _ in range(5)]


@pytest.mark.parametrize("keep,feat,p", [(0, torch.float32, 0.5), (1, torch.float32, 0.3),
                                         (1, torch.bfloat16, 0.5)])
def test_resume_is_bit_identical(csc, seq, keep, feat, p):
    say(f"checkpoint/resume keep={keep} feat={feat} p={p}")
    args = dict(n=2000, d=40, k=4, p=p, m=40, seed=113)
    kw = dict(lloyd_iters=10, keep_iterates=keep, feat_dtype=feat)
    Gs = [csc.Graph.from_workload(g) for g in seq]
    ref = csc.DynamicCSC(**args, **kw)
    ref_out = [ref.step(G) for G in Gs]
    a = csc.DynamicCSC(**args, **kw)
    for G in Gs[:3]:
        a.step(G)
    buf = a.export_state()
    h = csc.DynamicCSC.header(buf)
    assert h.t == 3 and h.n == 2000 and h.d == 40 and h.lam == ref_out[2][1]
    del a
    b = csc.DynamicCSC(**args, **kw)
    b.import_state(buf)
    for t in range(3, len(Gs)):
        lab, lam, r, cnt = b.step(Gs[t])
        assert torch.equal(lab, ref_out[t][0])
        assert (lam, r, cnt) == ref_out[t][1:]
    assert torch.equal(b.features(), ref.features())


def test_edited_cutoff_forces_refinement_as_in_oracle(csc, seq):
    say("edited lambda in the exported state")
    k, m, d, p, seed = 4, 40, 64, 0.5, 114
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32)
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10)
    for g in seq[:2]:
        orc.step(g)
        gpu.step(csc.Graph.from_workload(g))
    buf = gpu.export_state()
    csc.DynamicCSC.header(buf).lam = 1.9  # far above lambda_k: the fresh count is far above k
    gpu2 = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10)
    gpu2.import_state(buf)
    orc.lam = 1.9
    _, lam, ref, cnt = gpu2.step(csc.Graph.from_workload(seq[2]))
    r = orc.step(seq[2])
    say(f"  lam gpu={lam:.6f} oracle={r.lam:.6f}")
    assert ref and r.refined and lam < 1.9
    assert lam == r.lam
    assert cnt == pytest.approx(r.count, rel=1e-4, abs=1e-4)
    assert rel_fro(gpu2.features().double().cpu().numpy(), orc.theta) <= 1e-5


def test_state_errors(csc, seq):
    a = csc.DynamicCSC(2000, 40, 4, 0.5, 40, seed=115, keep_iterates=0)
    with pytest.raises(csc.CscError, match="CSC_E_STATE"):
        a.export_state()
    a.step(csc.Graph.from_workload(seq[0]))
    buf = a.export_state()
    other = csc.DynamicCSC(2000, 40, 4, 0.5, 40, seed=116, keep_iterates=0)
    with pytest.raises(csc.CscError, match="other parameters"):
        other.import_state(buf)
    bad = bytearray(buf)
    csc.DynamicCSC.header(bad).magic = 0
    with pytest.raises(csc.CscError, match="not a dynamic CSC state"):
        a.import_state(bad)
    with pytest.raises(csc.CscError, match="too small"):
        a.import_state(buf[:100])
