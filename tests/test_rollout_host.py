"""Host logic of the differentiable rollout: the choice between storing every
RK stage and checkpointing (no GPU needed)."""
import math

import pytest


@pytest.fixture(scope="module")
def AG():
    from paper_1810_11103_amd import autograd
    return autograd


def test_store_everything_when_it_fits(AG):
    # 400 steps of a 512^2 state (8 MiB): 3 x 400 x 8 MiB = 9.4 GiB
    sb = 4 * 512 * 512 * 8
    assert AG.choose_every(400, sb, 0.5, free_bytes=200 * 2**30) == 0
    assert AG.choose_every(400, sb, 0.5, free_bytes=3 * 400 * sb * 2) == 0


def test_checkpoint_spacing_minimises_memory_when_it_does_not(AG):
    sb = 4 * 512 * 512 * 8
    k = AG.choose_every(400, sb, 0.5, free_bytes=4 * 2**30)
    assert k == round(math.sqrt(400 / 3))
    # N/k + 3k is minimal at this spacing among integers
    cost = lambda e: math.ceil(400 / e) + 3 * e
    assert cost(k) <= min(cost(e) for e in range(1, 400)) + 1
    assert AG.choose_every(1, sb, 0.5, free_bytes=1) == 1
