"""The allocation-free labelling entry point (lbm_label_noalloc, static device scratch)
against lbm_label (caller workspace): identical labels, transport flags and counts, on two
calls in a row, the second on a smaller volume (the scratch keeps the first call's
contents and must be cleared), and the size limit."""
import sys

import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm
from paper_1410_1921_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_label_matches_workspace_label():
    torch.cuda.set_device(0)
    big, _, _ = lbm.lbm_reconstruct((96, 80, 112), 0.35, 7.0, 2.0, 1.0, 0.5, 0.5, 11)
    small = dev(W.random_mask((9, 17, 33), 0.4, 2))
    for pore in (big, small, big):
        say("shape", tuple(pore.shape))
        la, ta, sa = lbm.lbm_label(pore)
        lb, tb, sb = lbm.lbm_label_noalloc(pore)
        assert torch.equal(la, lb) and torch.equal(ta, tb)
        assert sa == sb
        say("components", sb["n_components"], "connectivity", sb["connectivity"])


def test_noalloc_label_limit():
    torch.cuda.set_device(0)
    pore = torch.zeros((257, 256, 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_label_noalloc(pore)
    assert e.value.status == lbm.LBM_E_NOMEM
    # the largest volume it takes
    m = dev(W.random_mask((256, 256, 256), 0.3, 5))
    la, ta, sa = lbm.lbm_label(m)
    lb, tb, sb = lbm.lbm_label_noalloc(m)
    assert torch.equal(la, lb) and torch.equal(ta, tb) and sa == sb
