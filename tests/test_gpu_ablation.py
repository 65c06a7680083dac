"""Encoder-design ablation (Sec. 3): every parallelisation encodes 32-bit words
into exactly the oracle's planes (block or register-block layout) and decodes
them back bit for bit, at sizes that leave ragged blocks, wavefronts and
2048-value regions."""
import numpy as np
import pytest

import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu

SIZES = [1, 31, 32, 33, 63, 64, 65, 2047, 2048, 2049, 100001, (1 << 20) + 5]


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


def _inputs(rng, n):
    yield rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    yield np.full(n, 0xFFFFFFFF, np.uint32)
    yield (np.arange(n, dtype=np.uint64) * 2654435761 % (2 ** 32)).astype(np.uint32)


@pytest.mark.parametrize("design", ["locality", "ballot", "shift", "butterfly", "regblock"])
def test_design_matches_oracle_and_round_trips(mdr, design):
    import torch
    rng = np.random.default_rng(13)
    for n in SIZES:
        for x in _inputs(rng, n):
            say("ablation", design, "n", n)
            ref = oracle.ablation_planes(x, design == "regblock")
            words = mdr.ablation_plane_words(design, n)
            assert ref.shape == (32, words)
            xd = torch.from_numpy(x.view(np.int32).copy()).cuda()
            planes = torch.full((32 * words,), -1, dtype=torch.int32, device="cuda")  # every word must be written
            mdr.ablation_encode(design, xd, planes)
            got = planes.cpu().numpy().view(np.uint32).reshape(32, words)
            assert np.array_equal(got, ref), (design, n)
            out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            mdr.ablation_decode(design, planes, out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), x), (design, n)


def test_rejects_misaligned_buffers(mdr):
    import torch
    x = torch.zeros(1000, dtype=torch.int32, device="cuda")
    planes = torch.zeros(32 * 64, dtype=torch.int32, device="cuda")
    with pytest.raises(mdr.MdrError) as ei:
        mdr.ablation_encode("locality", x[1:], planes)
    assert ei.value.status == mdr.MDR_ERR_INVALID_ARG
