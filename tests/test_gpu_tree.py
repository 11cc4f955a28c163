"""Invariants of the octree and the interaction lists the library builds on
the GPU (sec. 2.3: cells split while they hold ncrit or more Gauss points,
Eq. MAC for the far cells), read back through pbtc_get_tree:

* the children of every cell partition its sorted Gauss-point range and the
  leaves of every surface's tree partition that surface's range (each Gauss
  point in exactly one leaf); a leaf holds fewer than ncrit points;
* r_b of every cell is the largest distance from its centre to its points;
* every target group's bounding sphere holds its targets;
* for every (block, target group) item, its near and far cells cover the
  source surface's Gauss points exactly once (no point missed or counted
  twice), every far cell meets the MAC theta (|x_g - c| - r_g) > r_b with
  the group sphere, and every near cell is a leaf or a MAC-accepted cell
  with fewer sources than the block's P2P threshold.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which,theta,ncrit", [("star", 0.5, 0), ("multisurface", 0.6, 64)])
def test_tree_and_list_invariants(gpu_lib, which, theta, ncrit):
    from paper_1309_4018_amd import lib

    prob = synth.config2_star(nu=24, n_charges=300) if which == "star" else \
        synth.config3_multisurface(nu=12, cav_nu=6, n_charges=200)
    pl = lib.plan_for(prob, theta=theta, P=6, ncrit=ncrit)
    pl.setup()
    t = pl.tree()
    cells, gp, groups = t["cells"], t["gauss_points"], t["groups"]
    nc = len(cells)
    cx, cy, cz, half, rb = (cells[:, i] for i in range(5))
    begin, count, child, nchild = (cells[:, i].astype(np.int64) for i in range(5, 9))
    ncrit_eff = t["ncrit"]
    # children partition the parent's range
    for c in range(nc):
        if nchild[c] == 0:
            continue
        ch = np.arange(child[c], child[c] + nchild[c])
        assert begin[ch[0]] == begin[c]
        assert np.all(begin[ch[1:]] == begin[ch[:-1]] + count[ch[:-1]])
        assert begin[ch[-1]] + count[ch[-1]] == begin[c] + count[c]
    # leaves partition every surface's range; leaf sizes
    leaves = np.nonzero(nchild == 0)[0]
    assert np.all(count[leaves] < ncrit_eff) or ncrit_eff == 0
    for s, (g0, g1) in enumerate(t["surface_gp"]):
        lv = leaves[(begin[leaves] >= g0) & (begin[leaves] < g1)]
        lv = lv[np.argsort(begin[lv])]
        assert begin[lv[0]] == g0 and begin[lv[-1]] + count[lv[-1]] == g1
        assert np.all(begin[lv[1:]] == begin[lv[:-1]] + count[lv[:-1]])
    # r_b = max centre-point distance
    for c in range(nc):
        p = gp[begin[c]:begin[c] + count[c]]
        d = np.sqrt(((p - cells[c, :3]) ** 2).sum(axis=1)).max()
        assert abs(d - rb[c]) <= 1e-9 * max(d, 1.0)
    # group spheres hold their targets
    tg = t["targets"]
    for g, (gx, gy, gz, gr, t0, nt) in enumerate(groups):
        p = tg[int(t0):int(t0) + int(nt)]
        assert np.all(np.sqrt(((p - [gx, gy, gz]) ** 2).sum(axis=1)) <= gr * (1 + 1e-12) + 1e-12)
    # lists
    items = t["items"]  # (source root cell, group, P2P threshold, -)
    nptr, near, fptr, far = t["near_ptr"], t["near"], t["far_ptr"], t["far"]
    for it, (root, g, dbelow, _) in enumerate(items):
        gx, gy, gz, gr = groups[g, :4]
        nl = near[nptr[it]:nptr[it + 1]]
        fl = far[fptr[it]:fptr[it + 1]]
        allc = np.concatenate([nl, fl]).astype(np.int64)
        order = np.argsort(begin[allc])
        b, n = begin[allc][order], count[allc][order]
        assert b[0] == begin[root] and b[-1] + n[-1] == begin[root] + count[root], it
        assert np.all(b[1:] == b[:-1] + n[:-1]), it
        rtb_f = np.sqrt((gx - cx[fl]) ** 2 + (gy - cy[fl]) ** 2 + (gz - cz[fl]) ** 2) - gr
        assert np.all(theta * rtb_f > rb[fl]), it
        rtb_n = np.sqrt((gx - cx[nl]) ** 2 + (gy - cy[nl]) ** 2 + (gz - cz[nl]) ** 2) - gr
        ok = (nchild[nl] == 0) | ((theta * rtb_n > rb[nl]) & (count[nl] < dbelow))
        assert np.all(ok), it
