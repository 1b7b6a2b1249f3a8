"""Host logic of the launch-shape autotuner: which tile edges it tries
(those that divide every box side and whose fused-push LDS fits the 160 KB
of a gfx950 CU) and the LDS it counts for them (E on (T+3)^D cells, B on
(T+2)^D, the 8-byte current block on (T+3)^D, three components each)."""
import types

import pytest

from paper_1906_06306_amd import autotune


def box(D, n):
    return types.SimpleNamespace(D=D, n=n)


def test_lds_bytes_closed_forms():
    # 3D, edge 8, FP32: 3 (11^3 4 + 10^3 4 + 11^3 8) bytes
    assert autotune.lds_bytes(3, 8, 4) == 3 * (1331 * 4 + 1000 * 4 + 1331 * 8) == 59916
    # 3D, edge 16: 317 KB, beyond the CU's LDS
    assert autotune.lds_bytes(3, 16, 4) == 3 * (19 ** 3 * 4 + 18 ** 3 * 4 + 19 ** 3 * 8) == 316908
    # 2D, edge 32, FP64: 3 (35^2 8 + 34^2 8 + 35^2 8)
    assert autotune.lds_bytes(2, 32, 8) == 3 * (1225 * 8 + 1156 * 8 + 1225 * 8) == 86544
    assert autotune.lds_bytes(1, 16, 4) == 3 * (19 * 4 + 18 * 4 + 19 * 8)


@pytest.mark.parametrize("D,n,elem,want", [
    (2, (1024, 1024, 1), 4, [8, 16, 32]),     # the turbulence box
    (2, (1024, 1024, 1), 8, [8, 16, 32]),     # its FP64 path (T = 32: 86.5 KB)
    (3, (1024, 128, 128), 4, [8]),            # the shock box: 16^3 does not fit the LDS
    (2, (80, 48, 1), 4, [8, 16]),             # 32 divides neither side
    (2, (72, 40, 1), 4, [8]),
    (1, (512, 1, 1), 8, [8, 16, 32]),         # the two-stream box
    (2, (20, 12, 1), 4, []),                  # no edge divides both sides
])
def test_candidates(D, n, elem, want):
    assert autotune.candidates(box(D, n), elem) == want


def test_tune_refuses_a_box_without_candidates():
    with pytest.raises(ValueError, match="no tile edge"):
        autotune.tune(box(2, (20, 12, 1)), "fp32")
