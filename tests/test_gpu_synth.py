"""The device build of the input generator makes the same rows as the host
generator (inputs of the oracle always come from the host generator)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("index", ["zipf", "uniform"])
def test_device_rows_equal_host_rows(index):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    law = synth.RowLaw(synth.derive(77, synth.STREAM_DATA), 1 << 20, index=index)
    for row0, n in ((0, 20000), (123_456_789, 3000), (2**33 + 5, 100)):
        hip, hix = law.rows(row0, n)
        dip, dix = law.gpu_rows(row0, n)
        assert (dip.cpu().numpy() == hip).all()
        assert (dix.cpu().numpy() == hix).all()
