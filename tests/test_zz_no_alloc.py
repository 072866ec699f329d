"""x = M^T u through elmfb_rmatvec_noalloc (no device allocation: the chunk partials live in the
library's fixed scratch array) against elmfb_rmatvec (the handle's workspace), through the C
ABI: the same kernels, so the results are bit-identical; two calls in a row, the second on a
smaller problem (the array keeps the first call's contents, which must not leak into it); a
problem whose partials exceed the array is refused before any device work."""
import ctypes

import numpy as np
import pytest

from inputs import configs

from gpu_util import build, dev, torch_mod

pytestmark = pytest.mark.gpu


def _noalloc(P, u, x):
    from paper_2409_01949_amd import elmfb
    lib = elmfb.load_library()
    fn = lib.elmfb_rmatvec_noalloc
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_void_p] * 4
    torch = torch_mod()
    code = fn(P.h, u.data_ptr(), x.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if code != 0:
        msg = lib.elmfb_last_error(P.h)
        raise elmfb.ElmfbError(code, msg.decode() if msg else "")


def _compare(spec, seed):
    torch = torch_mod()
    P, W, b, f = build(spec)
    try:
        rows = P.sizes["n_rows"] + P.sizes["n_bc"]
        n = P.sizes["n_phi"]
        u = dev(np.random.default_rng(seed).standard_normal(rows))
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        got = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        P.rmatvec(u, ref)
        _noalloc(P, u, got)
        torch.cuda.synchronize()
        print(f"{spec.name}: {n} columns, max |diff| "
              f"{(got - ref).abs().max().item():.1e}")
        assert torch.equal(got, ref)
    finally:
        P.destroy()


def test_noalloc_matches_rmatvec_twice_then_smaller():
    # the larger problem first (3 levels, K = 20), then a smaller one (2 levels, K = 6), then the
    # oscillator, whose constraint rows enter the column pass
    _compare(configs.small2d(), 1)
    import dataclasses
    _compare(dataclasses.replace(configs.small2d(), name="tiny2d", n_points=(15, 13),
                                 levels=((1, 1), (2, 3)), K=6), 2)
    _compare(configs.oscillator(), 3)


def test_noalloc_refuses_beyond_its_scratch():
    """1,100 one-chunk subdomains with K = 256: 281,600 partials, more than the 262,144 the
    array holds: ELMFB_E_UNSUPPORTED, and the output is untouched."""
    from paper_2409_01949_amd import elmfb
    torch = torch_mod()
    spec = configs.tiny1d(K=256, J=1100, n=5000)
    P, W, b, f = build(spec)
    try:
        u = dev(np.ones(P.sizes["n_rows"]))
        x = torch.full((P.sizes["n_phi"],), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(elmfb.ElmfbError) as ei:
            _noalloc(P, u, x)
        assert ei.value.code == 6
        torch.cuda.synchronize()
        assert bool((x == 7.0).all())
    finally:
        P.destroy()
