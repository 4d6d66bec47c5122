"""Section 2's convergence stop on the GPU against the oracle: the same
number of rounds, bit-identical labels and centres, for several thresholds,
image shapes and launch variants."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth.configs import Workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


@pytest.mark.parametrize("w,h,S,threshold,variant", [
    (96, 72, 8, 0.05, 0), (96, 72, 8, 0.2, 1), (96, 72, 8, 1.0, 4), (96, 72, 8, 1e6, 0),
    (131, 57, 5, 0.3, 2), (640, 480, 16, 0.25, 0), (640, 480, 16, 0.25, 5), (64, 48, 8, 0.0, 0)])
def test_converge_matches_oracle(slic, w, h, S, threshold, variant):
    wl = Workload("conv", w, h, max(1, w * h // 500), 8.0, 7 + w, S)
    img = synth.image_for(wl)
    lab = oracle.rgb_to_lab(img)
    want_lb, want_cen, want_cnt, want_n = oracle.kmeans_converge(lab, S, 10.0, True, 15, threshold)
    p = slic.Params(w, h, S=S, m=10.0)
    slic.slic_set_assign_variant(w, h, S, variant)  # 0: the built-in choice
    try:
        ctx = slic.Context(p, torch.from_numpy(img.reshape(-1)).cuda())
        n = ctx.iterate_converge(15, threshold)
        lb = ctx.labels()
        cen, cnt = ctx.centres()
        e = ctx.energy()
        torch.cuda.synchronize()
        assert int(n.cpu()[0]) == want_n
        assert np.array_equal(lb.cpu().numpy(), want_lb)
        assert np.array_equal(cen.cpu().numpy(), want_cen)
        assert np.array_equal(cnt.cpu().numpy(), want_cnt)
        assert float(e.cpu()[0]) == pytest.approx(oracle.energy(lab, S, 10.0, want_cen, want_lb),
                                                  rel=1e-9)
        with pytest.raises(slic.SlicError):
            ctx.iterate(1)
        ctx.close()
    finally:
        slic.slic_set_assign_variant(w, h, S, 0)
