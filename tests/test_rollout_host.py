"""Host logic of the checkpoint driver: the automatic checkpoint interval."""
import math

import pytest

from paper_1809_02390_amd.rollout import choose_every, rollout_bytes

SB, AB = 9 * 512 * 512 * 4, 11 * 512 * 512 * 4  # state and adjoint bytes of a 512^2 lattice


def test_rollout_bytes_counts_checkpoints_pool_and_adjoints():
    assert rollout_bytes(2000, 1, SB, AB) == 2001 * SB + 2 * AB
    assert rollout_bytes(2000, 100, SB, AB) == (20 + 1 + 2 * 99 + 2) * SB + 2 * AB
    assert rollout_bytes(7, 2, SB, AB) == (4 + 1 + 2 * 1 + 2) * SB + 2 * AB
    assert rollout_bytes(50, 100, SB, AB) == (1 + 1 + 99) * SB + 2 * AB  # one segment: one set


def test_every_state_kept_when_it_fits():
    assert choose_every(2000, SB, AB, free_bytes=2 * rollout_bytes(2000, 1, SB, AB)) == 1


def test_square_root_interval_otherwise():
    free = 2 * rollout_bytes(2000, 45, SB, AB)
    assert free < rollout_bytes(2000, 1, SB, AB)
    assert choose_every(2000, SB, AB, free_bytes=free) == math.ceil(math.sqrt(2000))


def test_too_large_rejected():
    with pytest.raises(ValueError, match="GiB"):
        choose_every(10 ** 6, SB, AB, free_bytes=SB)
