import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def cfg1_setup():
    """Smallest workload: N=2048 uniform in the unit square, Matern-3/2 l=0.5,
    degree <= 1 (m=3), leaf 16, eta=1.6, |entries| < 1e-6 dropped."""
    import numpy as np

    import synth
    from oracle import compress, pattern, samplets, tree

    pts = synth.points_cube(2048, 2, 1)
    tr = tree.build_tree(pts, 16)
    b = samplets.build_samplets(tr, 1)
    blocks = pattern.block_pattern(tr, 1.6)
    rp, col = pattern.entry_csr(b, blocks)
    ks = compress.compress_dense(b, 1, 0.5, 1.0 / 2048)
    mask_prior = pattern.dense_mask(rp, col, 2048)
    mask_post = pattern.threshold_mask(mask_prior, ks, 1e-6)
    return dict(points=pts, tree=tr, basis=b, blocks=blocks, rp=rp, col=col, ks=ks,
                mask_prior=mask_prior, mask_post=mask_post, n=2048)
