"""The counter-calibration probe reads every byte of its buffer once: its sums
equal the host's, as dwords and as bytes, on sizes with ragged tails."""
import numpy as np
import pytest
import torch

import paper_2601_01787_amd as pmsz

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [4, 1020, 1 << 20, (1 << 24) + 12])
def test_probe_sums_every_byte_once(nbytes):
    rng = np.random.default_rng(nbytes)
    host = rng.integers(0, 256, size=nbytes, dtype=np.uint8)
    buf = torch.from_numpy(host).to("cuda:0")
    assert pmsz.probe_read(buf, 1) == int(host.astype(np.uint64).sum())
    assert pmsz.probe_read(buf, 0) == int(host.view(np.uint32).astype(np.uint64).sum())


def test_probe_rejects_bad_arguments():
    buf = torch.zeros(6, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(pmsz.PmszError):
        pmsz.probe_read(buf, 0)  # not a multiple of 4 bytes
    with pytest.raises(pmsz.PmszError):
        pmsz.probe_read(buf, 2)
