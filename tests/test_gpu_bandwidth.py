"""The attainable-bandwidth probe (lj_measure_bandwidth_shape) runs at the
launch shapes the ceiling sweep uses, including a vector length that is not
a whole number of rounds (the kernels skip the elements past the end), and
returns finite positive rates below twice the HBM peak (the probe's vectors
are four times its 64 MiB minimum; no expected values: a measurement)."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(256, 256, 4, True), (1024, 256, 1, False), (4096, 1024, 2, True)])
def test_bandwidth_probe_shapes(shape):
    import paper_2211_08948_amd as lj
    blocks, threads, unroll, nt = shape
    nbytes = (256 << 20) + 16 * 12345  # 256 MiB plus a ragged tail
    bw = lj.lj_measure_bandwidth_shape(nbytes, blocks, threads, unroll, nt)
    print("[case] bandwidth", shape, bw, flush=True)
    for k in ("copy", "read", "newton_step"):
        assert math.isfinite(bw[k]) and 0.0 < bw[k] < 16000.0
