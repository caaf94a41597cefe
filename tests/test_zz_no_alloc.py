"""The no-allocation QR entry point, rgs_qr_noalloc, against rgs_qr.

rgs_qr_noalloc runs the kernels of rgs_qr (Algorithm 2, Sec. 2.3) in the
library's fixed per-device scratch array instead of the handle's arena, with
step 1 on the handle's stream only and the P-SRHT rows drawn on the device.
Its Q, R and S must equal rgs_qr's bit for bit (the same arithmetic in the
same order; rgs_qr itself is held to the oracle by the other QR tests), on
two calls in a row, the second smaller than the first (the shared array
keeps the first call's contents), for every sketch and precision; also when
the fixed array forces step 1 into more, smaller column chunks than rgs_qr
uses.  Sizes beyond the array and flags are rejected before any device work.
"""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rgs():
    import paper_2011_05090_amd as rgs
    return rgs


def _inputs(n, m, k, prec, tag):
    rgs = _rgs()
    dt = torch.float64 if prec == "fp64" else torch.float32
    W = rgs.colmajor(n, m, dt)
    W.copy_(torch.from_numpy(synth.svd_matrix(n, m, 1e-3, tag=tag)))
    return W


def _outputs(n, m, k, prec):
    rgs = _rgs()
    dq = {"fp64": torch.float64, "fp32": torch.float32, "bf16q": torch.bfloat16}[prec]
    Q = rgs.colmajor(n, m, dq)
    Q.fill_(float("nan"))
    R = rgs.colmajor(m, m, torch.float64)
    R.fill_(float("nan"))
    S = rgs.colmajor(k, m, torch.float64)
    S.fill_(float("nan"))
    return Q, R, S


def _both(h, n, m, k, sketch, prec, tag, seed=11):
    rgs = _rgs()
    print("rgs_qr_noalloc vs rgs_qr: n %d m %d k %d %s %s" % (n, m, k, sketch, prec), flush=True)
    W = _inputs(n, m, k, prec, tag)
    d = rgs.qr_desc(n, m, k, sketch=sketch, prec=prec, seed=seed)
    Q0, R0, S0 = _outputs(n, m, k, prec)
    rep0 = rgs.rgs_qr(h, d, W, Q0, R0, S0)
    Q1, R1, S1 = _outputs(n, m, k, prec)
    rep1 = rgs.rgs_qr_noalloc(h, d, W, Q1, R1, S1)
    torch.cuda.synchronize()
    assert rep0.status == 0 and rep1.status == 0
    assert rep1.iters == m and rep1.failed_column == -1
    for a, b in ((Q0, Q1), (R0, R1), (S0, S1)):
        assert torch.equal(a, b)


CASES = [("srht", "fp64"), ("srht", "fp32"), ("srht", "bf16q"), ("gaussian", "fp64"), ("gaussian", "fp32"),
         ("gaussian", "bf16q"), ("rademacher", "fp32")]


@pytest.mark.parametrize("sketch,prec", CASES)
def test_noalloc_equals_rgs_qr_two_calls(gpu_handle, sketch, prec):
    # first call: fused projection + sketch pass (n >= 2^20 rows), ragged last block
    _both(gpu_handle, (1 << 20) + 333, 40, 256, sketch, prec, tag=301)
    # second, smaller call on the same array: split sketch path for the dense sketches
    _both(gpu_handle, 20011, 12, 64, sketch, prec, tag=302)


@pytest.mark.parametrize("sketch", ["srht", "gaussian"])
def test_noalloc_small_step1_chunks(gpu_handle, sketch):
    # k = 2048, m = 200: the fixed array leaves room for fewer step-1 columns per
    # chunk (about 48) than rgs_qr takes (64); the chunks run just before the
    # columns that read them
    _both(gpu_handle, (1 << 18) + 123, 200, 2048, sketch, "fp32", tag=303)


def test_noalloc_rejects_before_device_work(gpu_handle):
    rgs = _rgs()
    W = _inputs(4096, 8, 64, "fp32", 304)
    Q, R, S = _outputs(4096, 8, 64, "fp32")
    for flags in (rgs.FLAG_DIAGNOSTICS, rgs.FLAG_TIME_KERNELS, rgs.FLAG_CERTIFY):
        d = rgs.qr_desc(4096, 8, 64, sketch="gaussian", prec="fp32", flags=flags)
        with pytest.raises(rgs.RgsError) as e:
            rgs.rgs_qr_noalloc(gpu_handle, d, W, Q, R, S)
        assert e.value.status == rgs.RGS_EINVAL
    # P-SRHT rows beyond the device draw's limit
    n, m, k = 1 << 14, 4, 8192
    W = _inputs(n, m, k, "fp32", 305)
    Q, R, S = _outputs(n, m, k, "fp32")
    with pytest.raises(rgs.RgsError) as e:
        rgs.rgs_qr_noalloc(gpu_handle, rgs.qr_desc(n, m, k, sketch="srht", prec="fp32"), W, Q, R, S)
    assert e.value.status == rgs.RGS_ESCRATCH
    # sketch-space matrices beyond the array: five k x m fp64 matrices of 8 MiB each at
    # k = 4096, m = 256 fit; m = 512 (5 x 16 MiB) does not
    n, k = 8192, 4096
    for m, want in ((512, rgs.RGS_ESCRATCH), (256, rgs.RGS_OK)):
        W = torch.zeros((m, n), dtype=torch.float32, device="cuda").t()
        W.copy_(torch.randn(n, m, generator=torch.Generator().manual_seed(m)))
        Q, R, S = _outputs(n, m, k, "fp32")
        d = rgs.qr_desc(n, m, k, sketch="gaussian", prec="fp32")
        if want == rgs.RGS_OK:
            assert rgs.rgs_qr_noalloc(gpu_handle, d, W, Q, R, S).status == 0
        else:
            with pytest.raises(rgs.RgsError) as e:
                rgs.rgs_qr_noalloc(gpu_handle, d, W, Q, R, S)
            assert e.value.status == want
    torch.cuda.synchronize()
