"""The single-layer entry point that allocates nothing (stokes_sl_eval_noalloc), through
the C ABI, against stokes_sl_eval: FP64 to 1e-12 relative L2, mixed to 2e-6 relative
max-norm, on two calls in a row (the second smaller, so the static scratch holds the
first call's contents), on a problem whose partials need fewer source chunks than
stokes_sl_eval takes, with accumulation, and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1602_05650_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05650_amd import stokes
    return stokes


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _args(fs):
    return dict(src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length), eps=fs.eps)


def _compare(S, x, f, kw, mixed):
    ref = S.sl_eval(x, f, mixed=mixed, **kw).cpu().numpy()
    got = S.sl_eval_noalloc(x, f, mixed=mixed, **kw).cpu().numpy()
    e = rel_max(got, ref) if mixed else rel_l2(got, ref)
    assert e <= (2e-6 if mixed else 1e-12), e
    return e


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_two_calls_second_smaller(S, mixed):
    big = W.config1()["fibers"]          # 32,768 points
    small = W.config0()["fibers"]        # 512 points
    fb = np.random.default_rng(11).standard_normal((3, big.n))
    fs = np.random.default_rng(12).standard_normal((3, small.n))
    e1 = _compare(S, dev(big.xyz), dev(fb), _args(big), mixed)
    e2 = _compare(S, dev(small.xyz), dev(fs), _args(small), mixed)
    # explicit targets with a same-fiber exclusion, after the others
    trg = big.xyz[:, ::7]
    kw = dict(_args(big), trg_xyz=dev(trg), trg_fiber=dev(big.fiber[::7], torch.int32), excl="fiber")
    e3 = _compare(S, dev(big.xyz), dev(fb), kw, mixed)
    print(f"mixed={mixed}: {e1:.2e} {e2:.2e} {e3:.2e}")


def test_noalloc_fewer_chunks_and_accumulate(S):
    c = W.config2()                      # 262,144 points: the standard partials need 384 MiB
    fs = c["fibers"]
    x, f, kw = dev(fs.xyz), dev(c["force"]), _args(fs)
    for mixed in (True, False):
        _compare(S, x, f, kw, mixed)
    base = np.random.default_rng(13).standard_normal((3, fs.n))
    out = dev(base)
    S.sl_eval_noalloc(x, f, mixed=True, accumulate=True, out=out, **kw)
    ref = S.sl_eval(x, f, mixed=True, **kw).cpu().numpy()
    assert rel_max(out.cpu().numpy() - base, ref) <= 2e-6


def test_noalloc_rejects_what_does_not_fit(S):
    n = 600_000
    x = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    x[0] = torch.arange(n, dtype=torch.float64, device="cuda")
    f = torch.ones((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(S.StokesError) as ei:
        S.sl_eval_noalloc(x, f, excl=None, mixed=True)
    assert ei.value.code == S.E_INVAL
    assert "static scratch" in str(ei.value)
    # a diagnostics-free call is fine; the input scan is refused
    with pytest.raises(S.StokesError) as ei:
        S._check(S._lib.stokes_sl_eval_noalloc(2, S._ptr(x[:, :2].contiguous()), S._ptr(f[:, :2].contiguous()),
                                               None, None, 0, None, 2, None, None, None, 1.0, 0.01, 0.0,
                                               S.CHECK_INPUTS, S._ptr(f[:, :2].contiguous()), None))
    assert ei.value.code == S.E_INVAL
