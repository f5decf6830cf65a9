"""The register-resident butterfly microbenchmark (wally_diag_bfly_rate): its
arithmetic equals a Python model of the documented butterflies word for word,
and its rate is the measured peak of the transforms' butterfly on this chip."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

M32, M64 = (1 << 32) - 1, (1 << 64) - 1


def shoup4(a, w, wp, q):
    """The lazy Shoup product of the transforms: a w mod q in [0, 4q), with the
    quotient from three 32 x 32 partial products and the remainder formed mod
    2^64 through 2^64 - q."""
    a0, a1, p0, p1 = a & M32, a >> 32, wp & M32, wp >> 32
    mid = ((a0 * p1) >> 32) + ((a1 * p0) >> 32)
    qh = (a1 * p1 + mid) & M64
    h0, h1 = qh & M32, qh >> 32
    nq = (1 << 64) - q
    w0, w1, n0, n1 = w & M32, w >> 32, nq & M32, nq >> 32
    lo = (a0 * w0 + h0 * n0) & M64
    hi = ((lo >> 32) + a0 * w1 + a1 * w0 + h0 * n1 + h1 * n0) & M32
    return (hi << 32) | (lo & M32)


def csub(x, m):
    w = (x - m) & M64
    return x if w >> 63 else w


def model(tid, q, W, iters, inverse):
    x = [((tid * 16 + e) * 0x9E3779B97F4A7C15 & M64) % q for e in range(16)]
    q4 = 4 * q
    for _ in range(iters):
        for st in range(4):
            half = 8 >> st
            w, wp = W[st]
            for e in range(16):
                if e & half:
                    continue
                X, Y = x[e], x[e + half]
                if inverse:
                    u, v = (X + Y) & M64, (X - Y + q4) & M64
                    x[e], x[e + half] = csub(u, q4), shoup4(v, w, wp, q)
                else:
                    t = shoup4(Y, w, wp, q)
                    x[e], x[e + half] = (X + t) & M64, (X + q4 - t) & M64
    return x


@pytest.mark.parametrize("inverse", [0, 1])
@pytest.mark.parametrize("preset_name", ["tiny", "paper"])
def test_bfly_words_match_the_model(preset_name, inverse):
    from paper_2406_06761_amd.wally import Context, to_host

    c = Context.preset(preset_name)
    try:
        q, psi = c.info.q[0], c.info.psi[0]
        W = [(pow(psi, s + 1, q), (pow(psi, s + 1, q) << 64) // q) for s in range(4)]
        out = torch.zeros(2 * 256 * 16, dtype=torch.int64, device="cuda")
        bf, ms = c.bfly_rate(inverse, 2, 3, out)
        assert bf == 2 * 256 * 32 * 3 and ms > 0
        got = to_host(out).reshape(512, 16)
        for tid in (0, 1, 77, 255, 256, 511):
            assert [int(v) for v in got[tid]] == model(tid, q, W, 3, inverse), tid
        if inverse:  # the inverse butterflies keep words in [0, 4q)
            assert (got < np.uint64(4 * q)).all()
    finally:
        c.close()


def test_bfly_rate_is_near_the_issue_peak():
    """The measured forward and inverse rates on the paper's 54-bit prime; the
    peak derived from VALU issue (256 CUs x 64 lanes x 2.4 GHz / 20
    instructions per butterfly) is 1.966e12 per second."""
    from paper_2406_06761_amd.wally import Context

    c = Context.preset("paper")
    try:
        out = torch.empty(8192 * 256 * 16, dtype=torch.int64, device="cuda")
        for inverse in (0, 1):
            c.bfly_rate(inverse, 8192, 50, out)  # warm-up
            bf, ms = c.bfly_rate(inverse, 8192, 400, out)
            rate = bf / (ms * 1e-3)
            print(f"{'inverse' if inverse else 'forward'} butterflies: {rate:.4g} per second", flush=True)
            assert 0.3e12 < rate < 4e12
    finally:
        c.close()
