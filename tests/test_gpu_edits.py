"""The edit stream on the GPU (pmsz_encode_edits / pmsz_decode_edits) against
the oracle's encoder and decoder, byte for byte: synthetic changes of several
densities over more than one chunk, real corrections (halving and targeted)
in binary32 and binary64, the empty stream, and host-side rejection of
streams of another grid or cut short."""
import numpy as np
import pytest
import torch

import paper_2601_01787_amd as pmsz
import synth
from oracle import edits
from test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu


def _synthetic(dtype, n, frac, seed):
    rng = np.random.default_rng(seed)
    fhat = (rng.standard_normal(n) * 3).astype(dtype)
    g = fhat.copy()
    m = rng.uniform(size=n) < frac
    g[m] = (g[m].astype(np.float64) - rng.uniform(0, 1e-2, m.sum())).astype(dtype)
    g = np.minimum(g, fhat)
    return fhat.reshape(1, -1), g.reshape(1, -1)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("frac", [0.0, 0.001, 0.2, 1.0])
def test_stream_matches_oracle(dtype, frac):
    fhat, g = _synthetic(dtype, 40000, frac, 5)
    ref = edits.encode(fhat, g)
    s, ne = pmsz.encode_edits(dev(fhat), dev(g))
    assert ne == edits.parse_header(ref)["edits"]
    assert host(s).tobytes() == ref
    back = pmsz.decode_edits(dev(fhat), s)
    assert np.array_equal(host(back).view(np.uint8), g.view(np.uint8))
    # the GPU decoder reads the oracle's bytes too
    back2 = pmsz.decode_edits(dev(fhat), torch.from_numpy(np.frombuffer(ref, np.uint8).copy()).cuda())
    assert np.array_equal(host(back2).view(np.uint8), g.view(np.uint8))


@pytest.mark.parametrize("mode", ["halving", "targeted"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_stream_of_a_correction(mode, dtype):
    f, fhat, xi = synth.perlin_case(48, 4, 4, 1e-3, 21, dtype=torch.float32 if dtype == np.float32
                                    else torch.float64)
    f, fhat = f.cuda(), fhat.cuda()
    g, st = pmsz.correct(f, fhat, xi, mode=mode)
    assert st["status"] == "OK" and st["steps_applied"] > 0
    s, ne = pmsz.encode_edits(fhat, g)
    ref = edits.encode(host(fhat), host(g))
    assert host(s).tobytes() == ref
    assert ne == int(torch.count_nonzero(g != fhat))
    assert torch.equal(pmsz.decode_edits(fhat, s), g)


def test_bounded_workspace_reports_the_count():
    fhat, g = _synthetic(np.float32, 10000, 0.3, 9)
    n = int(np.count_nonzero(g != fhat))
    with pytest.raises(pmsz.PmszError) as e:
        pmsz.encode_edits(dev(fhat), dev(g), max_edits=n - 1)
    assert e.value.status == 6  # OOM
    s, ne = pmsz.encode_edits(dev(fhat), dev(g), max_edits=n)
    assert ne == n


def test_foreign_or_short_streams_are_rejected():
    fhat, g = _synthetic(np.float32, 5000, 0.1, 3)
    s, _ = pmsz.encode_edits(dev(fhat), dev(g))
    other = dev(np.zeros((1, 4000), np.float32))
    with pytest.raises(pmsz.PmszError):
        pmsz.decode_edits(other, s)                      # other grid
    with pytest.raises(pmsz.PmszError):
        pmsz.decode_edits(dev(fhat.astype(np.float64)), s)  # other type
    with pytest.raises(pmsz.PmszError):
        pmsz.decode_edits(dev(fhat), s[: s.numel() - 3].clone())  # cut short
