"""The entry point that allocates nothing (hd_point_distances_noalloc),
through the C ABI, against hd_point_distances: the same results bit for bit,
on two calls in a row (the second smaller, on scratch the first left behind),
in both arithmetics and both query kernels; the size limit is refused before
anything runs."""
import numpy as np
import pytest

from paper_2406_10357_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _hd():
    import torch
    import paper_2406_10357_amd as hd
    assert torch.cuda.is_available()
    hd.load_library()
    return hd, torch


@pytest.mark.parametrize("prec,lanes", [(0, 1), (1, 1), (0, 4), (1, 4)])
def test_noalloc_matches_point_distances(prec, lanes):
    hd, torch = _hd()
    W = wl.config(2, scale=0.1)
    rng = np.random.default_rng(7 + prec + lanes)
    lo, hi = W.VB.min(0), W.VB.max(0)
    P1 = np.concatenate([W.VA[rng.choice(W.VA.shape[0], 3000)], rng.uniform(lo - 0.2, hi + 0.2, size=(2000, 3))])
    P2 = rng.uniform(lo, hi, size=(1234, 3))
    print("[case] noalloc precision", prec, "lanes", lanes, "points", P1.shape[0], "then", P2.shape[0], flush=True)
    bvh = hd.build_bvh(torch.from_numpy(W.VB).cuda(), torch.from_numpy(W.FB).cuda())
    for P in (P1, P2):
        Pd = torch.from_numpy(P).cuda()
        d0, I0, Q0 = hd.point_distances(Pd, bvh, precision=prec, lanes=lanes)
        d1, I1, Q1, err = hd.point_distances_noalloc(Pd, bvh, precision=prec, lanes=lanes)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        assert torch.equal(d0, d1) and torch.equal(I0, I1) and torch.equal(Q0, Q1)


def test_noalloc_limit_and_arguments():
    hd, torch = _hd()
    W = wl.config(1)
    bvh = hd.build_bvh(torch.from_numpy(W.VB).cuda(), torch.from_numpy(W.FB).cuda())
    print("[case] noalloc limit", flush=True)
    too_many = torch.zeros((hd.NOALLOC_MAX_POINTS + 1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(hd.HDError) as e:
        hd.point_distances_noalloc(too_many, bvh)
    assert e.value.status == 2
    at_limit = torch.from_numpy(np.resize(W.VA, (hd.NOALLOC_MAX_POINTS, 3))).cuda()
    d0, I0, _ = hd.point_distances(at_limit, bvh)
    d1, I1, _, err = hd.point_distances_noalloc(at_limit, bvh)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and torch.equal(d0, d1) and torch.equal(I0, I1)
    none = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    _, _, _, err = hd.point_distances_noalloc(none, bvh)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
