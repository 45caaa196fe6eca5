"""Host-side checks of the post hoc helpers (no GPU): the per-block lattice
count is the lattice definition counted by brute force, block lattices of a
decomposition tile the domain lattice, and decompositions that do not split
into equal blocks of whole strides are refused before any device work."""

import numpy as np
import pytest


def test_lattice_count_is_the_definition():
    from paper_2004_02003_amd import posthoc

    for cells in range(1, 70):
        for stride in (1, 2, 3, 4):
            off = (stride - 1) / 2.0
            brute = sum(1 for m in range(cells + 2) if off + stride * m <= cells)
            assert posthoc.lattice_count(cells, stride) == brute, (cells, stride)


def test_block_lattices_tile_the_domain_lattice():
    from paper_2004_02003_amd import posthoc

    for stride in (1, 2, 3, 4):
        for blocks in (1, 2, 3, 4):
            cells = 12 * stride  # a whole number of strides per block
            per_block = posthoc.lattice_count(cells, stride)
            whole = posthoc.lattice_count(cells * blocks, stride)
            if stride == 1:
                # stride 1 puts seeds on the shared faces, which both neighbours own
                assert whole == per_block * blocks - (blocks - 1)
            else:
                assert whole == per_block * blocks


def test_run_blocks_refuses_uneven_decompositions():
    import torch
    from paper_2004_02003_amd import posthoc

    g = [torch.zeros((13, 13, 13, 3))]
    with pytest.raises(ValueError):
        posthoc.run_blocks(g, np.array([0.0]), (5, 1, 1), 2)   # 12 cells do not split into 5 blocks
    with pytest.raises(ValueError):
        posthoc.run_blocks(g, np.array([0.0]), (4, 1, 1), 2)   # 3 cells per block is not a whole stride
    with pytest.raises(ValueError):
        posthoc.run_blocks(g, np.array([0.0]), (2, 2, 2), 1)   # stride 1: face seeds in two blocks
