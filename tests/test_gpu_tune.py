"""The multi-state autotuner on the GPU: it writes a loadable cache, and the
operator stays at parity with the FP64 oracle under the tuned plans (the
tolerance of the on-the-fly parity tests)."""
import json
import math

import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def test_tune_writes_cache_and_keeps_parity(ctx, tmp_path):
    L = P.lib()
    path = tmp_path / "tune.json"
    try:
        P.tune(ctx, str(path), n_max=8192, B_max=16)
        data = json.loads(path.read_text())
        entries = data["entries"]
        assert {(e["npad"], e["B"]) for e in entries} == {(n, b) for n in (1024, 2048, 8192) for b in (2, 4, 16)}
        for e in entries:
            assert e["target_wgs"] in (256, 512, 1024, 2048, 4096) and e["ms"] > 0
            assert L.nfr_tune_target(e["npad"], e["B"]) == e["target_wgs"]
        L.nfr_tune_clear()
        P.tune_load(str(path))
        rng = np.random.default_rng(5)
        for n, B in ((2000, 4), (7000, 16), (1500, 2)):
            x = S.fibonacci_sphere(n)
            q = np.full(n, 4 * math.pi / n) * rng.uniform(0.9, 1.1, size=n)
            U = rng.normal(0.2, 0.4, size=(B, n))
            theta = rng.uniform(0.1, 0.3, size=B)
            p = (1.0, 0.15, 0.5, 0.4)
            prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
            y = prob.apply(P.kernel_struct(NF.GAUSS_MH, *p), P.Firing(20.0, torch.from_numpy(theta).cuda()),
                           torch.from_numpy(U).cuda()).cpu().numpy()
            ref = NF.apply_K(x, q, U, NF.GAUSS_MH, p, 20.0, theta)
            G = q[None, :] * NF.firing(U, 20.0, theta)
            scale = np.abs(G) @ np.abs(NF.kernel_matrix(x, NF.GAUSS_MH, p)).T
            assert np.max(np.abs(y - ref) / scale) <= 1e-5
    finally:
        L.nfr_tune_clear()
