"""Every storage form of the filter against its storage floor (Sec. 2.2, Step 1; eq.
static_filtering).

The floor of a form is the error of the FP64 recurrence rounded only where that form stores
values (oracle.storage).  A kernel that rounds at those points and nowhere else lands near
its floor; one that drops a term, rounds twice or loses the FP32 state lands far above it.
The output is taken in FP32 here (and emulated so), so that the floor is that of the operator
values and the iterates.  Two cases:
  * C1 (SBM N = 1000, k = 5, degree 16, ratio 0.1) at its cut-off midway between lambda_5
    and lambda_6, where the filter keeps 7% of the signals' norm;
  * an SBM of N = 20,000 nodes in 20 blocks (degree 16, ratio 0.1) at the cut-off 0.1, below
    its community eigenvalues, where the filter keeps 0.7%: the same absolute rounding is then
    a large fraction of the output, as at the C3 operating cut-off, and the 16-bit forms
    separate (BF16 iterates 4.8e-2 of the output, binary16 6.1e-3).
The bound is max(1e-5, 2 x floor) relative to the output, and every bound sits far enough
below 1 that an all-zero output fails.
"""

import numpy as np
import pytest
import torch

from oracle import chebyshev, operator, storage
from workloads import gaussian_block, sbm, seed_for
from helpers import rel_fro, say

pytestmark = pytest.mark.gpu

# GPU form -> (emulated form, iterate mode, signals and operator values)
FORMS = {
    "fp32": ("fp32_onepass", torch.float32, torch.float32),
    "bf16io": ("bf16io_onepass", torch.float32, torch.bfloat16),
    "bf16": ("bf16_onepass", torch.bfloat16, torch.bfloat16),
    "bf16s": ("bf16s_onepass", "bf16s", torch.bfloat16),
    "f16": ("f16_onepass", torch.float16, torch.bfloat16),
    "f16s": ("f16s_onepass", "f16s", torch.bfloat16),
}
M = 50


def _case(csc, g, lam_c):
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    X = gaussian_block(g.n, 64, 1 / np.sqrt(64), seed=10)
    return dict(g=g, A=A, lam_c=lam_c, X=X, G32=csc.Graph.from_workload(g),
                G16=csc.Graph.from_workload(g, val_dtype=torch.bfloat16), floors={})


@pytest.fixture(scope="module")
def cases(csc):
    g1 = sbm(1000, 5, 16.0, 0.1, seed=seed_for(1, "graph"))
    A1, _ = operator.normalized_adjacency(g1.n, g1.rowptr, g1.colidx, g1.w)
    lam = np.linalg.eigvalsh(np.eye(g1.n) - A1.toarray())
    return {"c1": _case(csc, g1, 0.5 * (lam[4] + lam[5])),
            "deep": _case(csc, sbm(20_000, 20, 16.0, 0.1, seed=91), 0.1)}


def _run(csc, c, form, variant):
    emu, iters, io = FORMS[form]
    a = chebyshev.step_coefficients(M, 2.0, c["lam_c"], "jackson")
    Xt = torch.from_numpy(c["X"]).cuda().to(io)
    Xin = Xt.double().cpu().numpy()
    G = c["G32"] if io == torch.float32 else c["G16"]
    G.set_variant(variant, iters)
    Y = csc.cheb_filter(G, a, Xt, out_dtype=torch.float32, iter_dtype=iters)
    G.set_variant(-1, iters)
    ref = chebyshev.filter_recurrence(c["A"], 2.0, a, Xin)
    if emu not in c["floors"]:
        Ye = storage.filter_stored(c["A"], 2.0, a, Xin, **dict(storage.FORMS[emu], out="f32"))
        c["floors"][emu] = rel_fro(Ye, ref)
    gain = np.linalg.norm(ref) / np.linalg.norm(Xin)
    return rel_fro(Y.double().cpu().numpy(), ref), c["floors"][emu], gain


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("case", ["c1", "deep"])
@pytest.mark.parametrize("form", list(FORMS))
def test_form_within_twice_its_floor(csc, cases, form, case, variant):
    c = cases[case]
    err, floor, gain = _run(csc, c, form, variant)
    bound = max(1e-5, 2.0 * floor)
    say(f"{form} {case} variant {variant} cut-off {c['lam_c']:.4f} (gain {gain:.4f}): "
        f"error {err:.3e}, floor {floor:.3e}, ratio {err / floor:.2f}")
    assert bound < 0.5  # an all-zero output (error 1) fails
    assert err <= bound


def test_half_forms_beat_bf16_at_the_deep_cut_off(csc, cases):
    """binary16 keeps three more significant bits than BF16 at the same two bytes: at the deep
    cut-off its error must be several times smaller, in the plain and in the split form."""
    c = cases["deep"]
    err = {f: _run(csc, c, f, -1)[0] for f in ("bf16", "f16", "bf16s", "f16s")}
    say(f"  deep cut-off errors {err}")
    assert err["f16"] * 4 < err["bf16"]
    assert err["f16s"] * 4 < err["bf16s"]
