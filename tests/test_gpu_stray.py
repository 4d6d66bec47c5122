"""Section 3's stray-pixel filter on the GPU against the oracle (exact), on
SLIC label maps and on noisy random maps, for 0..3 passes."""
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


@pytest.mark.parametrize("w,h,S,passes", [(160, 120, 16, 2), (131, 77, 8, 1), (97, 45, 5, 3),
                                          (640, 480, 16, 2), (1, 37, 4, 2), (53, 1, 4, 0)])
def test_stray_filter_matches_oracle(slic, w, h, S, passes):
    wl = Workload("stray", w, h, max(1, w * h // 500), 12.0, 700 + w, S)
    img = synth.image_for(wl)
    lab = oracle.rgb_to_lab(img)
    labels, _, _ = oracle.kmeans(lab, S, 10.0, True, 5)
    want = oracle.stray_filter(labels, passes)
    ctx = slic.Context(slic.Params(w, h, S=S, m=10.0), torch.from_numpy(img.reshape(-1)).cuda())
    ctx.iterate(5)
    got = ctx.filter_stray(passes).labels()
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    with pytest.raises(slic.SlicError):
        ctx.iterate(1)
    ctx.close()
