"""The batch's single cooperative persistent launch gives the same results as
the phased launches."""
import numpy as np
import pytest
import torch

from test_gpu_batch import check, make_frames

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_batch_cooperative_equals_phased(layout):
    import paper_1711_01656_amd as ih
    frames = make_frames(21, np.uint8, n=6)
    batch = ih.Batch(frames, "chi2", layout=layout)
    batch.run("cooperative")
    torch.cuda.synchronize()
    check(batch, frames, "chi2", layout)
    coop = [t.clone() for t in batch.ih]
    batch.run("phased")
    torch.cuda.synchronize()
    for a, b in zip(coop, batch.ih):
        assert torch.equal(a, b)
