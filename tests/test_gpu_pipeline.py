"""GPU parity of the chunked H2D / refactor / D2H pipeline: every chunk's
refactored container equals the oracle's for that chunk alone, and retrieval
through the pipeline (all planes, and a tolerance planned per chunk) writes to
host memory exactly the oracle's reconstructions; with and without overlap.
The retrieval uploads only the units each chunk's plan needs (its sign unit
and the groups below its planes), byte for byte what the oracle's plan reads."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_same_bits, say, to_oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdr():
    import paper_2505_00227_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mdr):
    c = mdr.Context(0)
    yield c
    c.close()


def _planned_unit_bytes(levels, k):
    """Bytes of the units that planes k need: each level's sign unit and every
    group whose first plane is below k (placeholders hold 0 bytes)."""
    total = 0
    for lv, kl in zip(levels, k):
        if kl == 0:
            continue
        total += len(lv.streams[0][1])
        for first in range(0, kl, lv.m):
            total += len(lv.streams[1 + first][1])
    return total


@pytest.mark.parametrize("dtype,B", [(np.float64, 64), (np.float64, 40), (np.float32, 32)])
def test_pipeline_matches_oracle_per_chunk(mdr, ctx, dtype, B):
    import torch
    sizes = workloads.chunk_level_sizes(slab=4, edge=32, nlevels=4)
    nchunks = 3
    chunks = [workloads.chunk_levels(seed=9, chunk=c, slab=4, edge=32, nlevels=4, dtype=dtype)
              for c in range(nchunks)]
    flat = np.concatenate([np.concatenate(ch) for ch in chunks])
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    host = torch.from_numpy(flat).pin_memory()
    out = torch.empty(flat.size, dtype=tdt).pin_memory()
    p = mdr.default_params()
    pipe = mdr.Pipeline(ctx, nchunks, sizes, tdt, B, p)
    op = to_oracle_params(p)
    orc = [oracle.refactor(ch, B, op) for ch in chunks]
    lo = min(float(a.min()) for ch in chunks for a in ch if a.size)
    hi = max(float(a.max()) for ch in chunks for a in ch if a.size)
    for overlap in (True, False):
        say("pipeline", dtype, B, "overlap", overlap)
        info = pipe.refactor(host, overlap=overlap)
        assert info["h2d_bytes"] == flat.nbytes
        for c in range(nchunks):
            assert pipe.chunk(c).serialize() == oracle.serialize(orc[c], op), ("chunk", c)
        # pinned output (written by a kernel through its device address) and
        # pageable output (copies); both start poisoned
        for pinned in (True, False):
            dst = out if pinned else torch.empty(flat.size, dtype=tdt)
            for rel in (0.0, 1e-4, 1e-2):
                dst.fill_(float("nan"))
                info = pipe.retrieve(rel, dst, relative=True, overlap=overlap)
                got = dst.numpy()
                o = 0
                want_h2d = 0
                for c in range(nchunks):
                    vals, k, bound, met = oracle.retrieve_to(orc[c], rel * (hi - lo), relative=False)
                    ref = np.concatenate(vals)
                    assert_same_bits(got[o:o + ref.size], ref, ("chunk", c, "rel", rel, "pinned", pinned))
                    o += ref.size
                    want_h2d += _planned_unit_bytes(orc[c], k)
                # progressive fetch: exactly the sign unit and the planned groups crossed PCIe
                assert info["h2d_bytes"] == want_h2d, (rel, info["h2d_bytes"], want_h2d)
