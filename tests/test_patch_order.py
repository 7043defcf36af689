"""Host logic of the fine-tuner's patch sampler (no GPU): every ray id
exactly once per epoch, grouped into whole 8x8 patches (ragged at image
edges), patches in a seeded order."""
import torch

import workloads as W
from paper_2103_14645_amd import finetune as F


class _Cams:
    """The attributes patch_order reads, without a device or a library handle."""

    def __init__(self, cams):
        self.cam_list = cams
        self.mlp = torch.zeros(1)


def test_patch_order_is_a_permutation_of_whole_patches():
    cams = [W.orbit_camera(20, 13, seed=1), W.orbit_camera(8, 8, seed=2), W.orbit_camera(5, 17, seed=3)]
    st = _Cams(cams)
    g = torch.Generator()
    g.manual_seed(0)
    ids = F.MlpFineTuner.patch_order(st, g)
    n = sum(c.W * c.H for c in cams)
    assert sorted(ids.tolist()) == list(range(n))
    # walk the order: each run of ids belongs to one patch of one camera
    offs = [0]
    for c in cams:
        offs.append(offs[-1] + c.W * c.H)

    def patch_of(r):
        ci = max(i for i in range(len(cams)) if offs[i] <= r)
        loc = r - offs[ci]
        return ci, (loc // cams[ci].W) // 8, (loc % cams[ci].W) // 8

    seen, prev, runs = set(), None, 0
    for r in ids.tolist():
        p = patch_of(r)
        if p != prev:
            assert p not in seen, "a patch appears in two places"
            seen.add(p)
            prev = p
            runs += 1
    assert runs == sum(((c.W + 7) // 8) * ((c.H + 7) // 8) for c in cams)
    g2 = torch.Generator()
    g2.manual_seed(0)
    assert torch.equal(F.MlpFineTuner.patch_order(st, g2), ids)  # seeded
