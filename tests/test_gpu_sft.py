"""GPU parity of the data preparation (Sec. 2): strain -> Hann-windowed
short Fourier transforms -> normalised power rho = P ln 2 / running median.

Bar, from the arithmetic: the transform is FP32, so each |X_k| carries an
absolute error of order eps_32 log2(N) times the spectrum's rms; rho = P ln2 /
median then differs from the FP64 oracle by at most 2e-5 (1 + rho) here.  The
running median is an order statistic: a swap of two nearly equal powers moves
it by no more than their difference, so it stays within the same bound.
Cases: noise with a bin-centred line, ragged band ends (not multiples of the
256-bin tile), the widest (257) and narrowest (1) windows, a band that
touches both limits (k_lo = window/2 and the Nyquist bin), several chunks of
segments, zero strain (rho = 0) and the error paths.
"""
import numpy as np
import pytest

from oracle import sft

pytestmark = pytest.mark.gpu


def _run(x, n_fft, k_lo, n_bins, window):
    import torch
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    try:
        rho = ctx.sft_normalise(torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda(), n_fft, k_lo,
                                n_bins, window)
        return rho.cpu().numpy().astype(np.float64)
    finally:
        ctx.close()


def _check(x, n_fft, k_lo, n_bins, window, tol=2e-5):
    got = _run(x, n_fft, k_lo, n_bins, window)
    want = sft.normalised_power(np.asarray(x, np.float32), n_fft, k_lo, n_bins, window)
    assert got.shape == want.shape
    err = np.abs(got - want) / (1.0 + want)
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))
    return got, want


@pytest.mark.parametrize("n_fft,n_seg,k_lo,n_bins,window", [
    (4096, 40, 300, 1200, 101),
    (4096, 7, 200, 1000, 257),      # the widest window, a ragged last tile
    (1024, 5, 128, 257, 1),         # window 1: rho = ln 2 everywhere
    (512, 3, 50, 157, 101),         # band reaching the Nyquist bin: 50 + 156 + 50 = 256
    (256, 9, 0, 129, 1),            # k_lo = 0 with window 1, up to Nyquist
])
def test_noise_against_oracle(n_fft, n_seg, k_lo, n_bins, window):
    print(f"case: sft n_fft={n_fft} n_seg={n_seg} k_lo={k_lo} n_bins={n_bins} window={window}", flush=True)
    r = np.random.default_rng(n_fft + n_seg)
    x = r.normal(0.0, 3.0, n_fft * n_seg).astype(np.float32)
    got, want = _check(x, n_fft, k_lo, n_bins, window)
    if window == 1:
        assert np.allclose(got, np.log(2.0), rtol=1e-6)
    else:
        assert 0.9 < got.mean() < 1.1


def test_line_stands_out():
    n_fft, n_seg = 8192, 12
    r = np.random.default_rng(63)
    n = np.arange(n_fft * n_seg)
    # line power (A N/4)^2 = 1.7e5 against the noise mean 3N/8 = 3.1e3: rho ~ 55
    x = (r.normal(size=n.size) + 0.2 * np.cos(2 * np.pi * 2000 * n / n_fft)).astype(np.float32)
    got, want = _check(x, n_fft, 1500, 1000, 101)
    assert np.all(got[:, 500] > 20.0)        # bin 2000 carries the line in every segment
    assert np.all(np.argmax(got, axis=1) == 500)


@pytest.mark.slow
def test_many_chunks_realistic_segment_length():
    """8-s segments at 4096 Hz (32768 samples): 4200 segments span two chunks
    of the library's spectra buffer (4095 segments, then a ragged 105); a
    narrow band keeps the oracle quick.  The strain is only read: unchanged
    after two calls, which agree bit for bit."""
    import torch
    from paper_2507_07816_amd import ltgw

    print("case: sft 4200 x 32768", flush=True)
    n_fft, n_seg = 32768, 4200
    r = np.random.default_rng(64)
    x = r.normal(size=n_fft * n_seg).astype(np.float32)
    ctx = ltgw.Context(0)
    try:
        dev = torch.from_numpy(x).cuda()
        keep = dev.clone()
        a = ctx.sft_normalise(dev, n_fft, 4000, 300, 101)
        b = ctx.sft_normalise(dev, n_fft, 4000, 300, 101)
        assert torch.equal(dev, keep)
        assert torch.equal(a, b)
        got = a.cpu().numpy().astype(np.float64)
    finally:
        ctx.close()
    del dev, keep
    want = sft.normalised_power(x, n_fft, 4000, 300, 101)
    err = np.abs(got - want) / (1.0 + want)
    assert err.max() <= 2e-5, (err.max(), np.unravel_index(err.argmax(), err.shape))


def test_zero_strain_and_errors():
    import torch
    from paper_2507_07816_amd import ltgw

    assert np.array_equal(_run(np.zeros(1024 * 3), 1024, 100, 200, 51), np.zeros((3, 200)))
    ctx = ltgw.Context(0)
    E = ltgw.LtgwError
    x = torch.zeros(1024 * 3, dtype=torch.float32, device="cuda")
    out = torch.empty((3, 200), dtype=torch.float32, device="cuda")
    try:
        for args in [(3, 1024, 100, 200, 50), (3, 1024, 100, 200, 259), (3, 1024, 20, 200, 51),
                     (3, 1024, 400, 200, 51), (3, 1023, 100, 200, 51), (0, 1024, 100, 200, 51)]:
            with pytest.raises(E) as ei:
                ltgw.ltgw_sft_normalise(ctx.h, x, *args, out)
            assert ei.value.code == ltgw.LTGW_E_INVALID_ARG, args
        with pytest.raises(E) as ei:
            ltgw.ltgw_sft_normalise(ctx.h, np.zeros(3072, np.float32), 3, 1024, 100, 200, 51, out)
        assert ei.value.code == ltgw.LTGW_E_INVALID_ARG
        ltgw.ltgw_sft_normalise(ctx.h, x, 3, 1024, 100, 200, 51, out)
        assert float(out.abs().max()) == 0.0
    finally:
        ctx.close()


def test_strain_is_not_written():
    """The transform works on a copy of the caller's strain: a second call on
    the same strain gives the same rho, and the strain is unchanged."""
    import torch
    from paper_2507_07816_amd import ltgw

    r = np.random.default_rng(65)
    x = r.normal(size=8192 * 6).astype(np.float32)
    ctx = ltgw.Context(0)
    try:
        dev = torch.from_numpy(x).cuda()
        a = ctx.sft_normalise(dev, 8192, 1000, 2000, 101).cpu().numpy()
        b = ctx.sft_normalise(dev, 8192, 1000, 2000, 101).cpu().numpy()
        assert np.array_equal(dev.cpu().numpy(), x)
        assert np.array_equal(a, b)
    finally:
        ctx.close()
