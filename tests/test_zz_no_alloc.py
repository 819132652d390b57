"""The entry point that allocates nothing: ddx_tree_dedisperse_static against
ddx_tree_dedisperse with a caller-owned workspace (same kernels, so bitwise equal),
on two calls in a row, the second smaller, and the size limit."""
import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_static_workspace_matches_workspace_argument(gpu):
    import torch

    from paper_1109_3186_amd import ESIZE, DdxError, TREE_STATIC_MAX, tree_dedisperse, tree_dedisperse_static
    g = torch.Generator(device=gpu)
    g.manual_seed(1115)
    for c, t in [(256, 40000), (64, 9001)]:  # the second call is smaller
        power = torch.rand((c, t), dtype=torch.float32, device=gpu, generator=g)
        ref = tree_dedisperse(power, out=torch.empty_like(power), work=torch.empty_like(power))
        got = tree_dedisperse_static(power, torch.full_like(power, float("nan")))
        torch.cuda.synchronize()
        same = bool(torch.equal(got, ref))
        say("static workspace, %d channels x %d samples: bitwise equal %s" % (c, t, same))
        assert same
    big = torch.empty((1024, TREE_STATIC_MAX // 1024 + 1), dtype=torch.float32, device=gpu)
    with pytest.raises(DdxError) as e:
        tree_dedisperse_static(big, torch.empty_like(big))
    assert e.value.status == ESIZE
