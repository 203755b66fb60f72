"""The five workload configurations, as plain data.

C1  static SBM  N=1,000,    k=5,   degree 16, ratio 0.1, d=32,  m=50,  lambda_c from dense eigh
C2  static SBM  N=200,000,  k=20,  degree 20, ratio 0.1, d=64,  m=100, 24 probes, 16 bisection steps
C3  dynamic SBM N=1,000,000, k=50 Zipf(1.2) sizes, degree 16, T=20, 1% edges rewired and
    0.5% nodes moved per snapshot, d=128, m=120, p=0.5
C4  adjoint     N=200,000,  k=20,  degree 20, d=64,  m=60, checkpoint every 8 iterates;
    gradcheck graph N=2,000, k=4, degree 10
C5  Chung-Lu    N=8,000,000, 200 communities, exponent 2.5, degree 20, T=10, 0.5% rewired,
    d=256, m=150, p=0.75
"""

from __future__ import annotations


def config_seed(config: int) -> int:
    return 20170603 + 100 * int(config)


CONFIGS = {
    1: dict(n=1000, k=5, degree=16.0, ratio=0.1, d=32, m=50, lloyd=20, sizes="equal"),
    2: dict(n=200_000, k=20, degree=20.0, ratio=0.1, d=64, m=100, n_probe=24, n_cand=16,
            sizes="equal"),
    3: dict(n=1_000_000, k=50, degree=16.0, ratio=0.1, d=128, m=120, p=0.5, T=20,
            rewire=0.01, move=0.005, sizes="zipf", zipf_s=1.2, lloyd=20, n_cand=16),
    4: dict(n=200_000, k=20, degree=20.0, ratio=0.1, d=64, m=60, ckpt=8,
            small=dict(n=2000, k=4, degree=10.0, ratio=0.1)),
    5: dict(n=8_000_000, k=200, degree=20.0, ratio=0.1, exponent=2.5, d=256, m=150, p=0.75,
            T=10, rewire=0.005, lloyd=20, n_cand=16),
}
