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


@pytest.mark.parametrize("layout", ["bhw", "hwb"])
def test_batch_cooperative_64_uneven_frames(layout):
    """The benchmark's 64 uneven frames (4,096 candidates each): the
    cooperative launch's histograms, distances and best candidates equal the
    phased launches', which the oracle checks in test_batch_64_uneven_frames."""
    import paper_1711_01656_amd as ih
    import synth
    print("64 uneven frames, cooperative vs phased", layout, flush=True)
    frames = [dict(img=torch.from_numpy(f.img).cuda(), bins=f.bins, value_bits=f.bits,
                   origins=torch.from_numpy(f.origins).cuda(), win=(32, 32), tmpl_win=f.tmpl_win)
              for f in synth.config4()]
    batch = ih.Batch(frames, "chi2", layout=layout)
    batch.run("phased")
    torch.cuda.synchronize()
    ref = [t.clone() for t in batch.ih]
    ref_d = [t.clone() for t in batch.dist]
    ref_b = [t.clone() for t in batch.best]
    for t in batch.ih:
        t.fill_(-1)
    batch.run("cooperative")
    torch.cuda.synchronize()
    for i in range(len(frames)):
        assert torch.equal(batch.ih[i], ref[i]), i
        assert torch.equal(batch.dist[i], ref_d[i]), i
        assert torch.equal(batch.best[i], ref_b[i]), i


def test_cooperative_batch_refuses_graph_capture():
    """Under stream capture the cooperative mode returns an error before
    enqueuing anything (a captured cooperative launch would lose its
    co-residency guarantee); the phased mode of the same batch captures."""
    import paper_1711_01656_amd as ih
    frames = make_frames(23, np.uint8, n=4)
    batch = ih.Batch(frames, "chi2", layout="bhw")
    batch.run("phased")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with pytest.raises(ih.IHError, match="cannot be captured"):
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                batch.run("cooperative")
    torch.cuda.synchronize()
    batch.run("cooperative")                      # eager: still runs, same results
    torch.cuda.synchronize()
    check(batch, frames, "chi2", "bhw")
