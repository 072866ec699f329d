"""The learned warm start end to end at reduced size (1,024 training solves, 256 held out): the
batched solver generates the training data, the library's MLP is trained on it, and held-out
solves started from its prediction meet the same FP64 residual target as cold solves in fewer
iterations.  The oracle judges the warm solutions' residuals on a sample of pairs."""
import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm

from gpu_util import torch_mod

pytestmark = pytest.mark.gpu


def test_learned_warm_start_gains():
    torch = torch_mod()
    from paper_2409_01949_amd import warmstart as ws

    om, C = configs.warm_groups(128, 5)
    B, specs, _ = ws.family_batch(om, C)
    coef, infos, t_data = ws.solve_batch(B, btol=1e-5, inner=2000, outer=6)
    X, F = ws.family_inputs(specs, om, C)
    Y = ws.coef_blocks(coef, specs, C.shape[1])
    B.destroy()
    W = ws.WarmStart(n_in=X.shape[1], K=Y.shape[1], max_batch=4096, seed=0)
    hist = W.fit(X, F, Y, epochs=100, lr=1e-3, seed=0)
    print(f"data {t_data:.1f} s; loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.5 * hist[0]

    om2, C2 = configs.warm_groups(32, 6)
    B2, specs2, hn2 = ws.family_batch(om2, C2)
    X2, F2 = ws.family_inputs(specs2, om2, C2)
    pred = W.predict(X2, F2)
    x0 = torch.as_tensor(np.ascontiguousarray(pred).reshape(-1)).cuda()
    btol = 1e-4
    _, cold, tc = ws.solve_batch(B2, btol=btol, inner=2000, outer=8)
    yw, warm, tw = ws.solve_batch(B2, x0=x0, btol=btol, inner=2000, outer=8, precondition=False)
    itc = np.array([i["iters"] for i in cold])
    itw = np.array([i["iters"] for i in warm])
    print(f"held-out: cold {tc:.2f} s, mean iters {itc.mean():.0f} (max {itc.max()}); "
          f"warm {tw:.2f} s, mean iters {itw.mean():.0f} (max {itw.max()})")
    assert all(i["istop"] == 1 for i in cold) and all(i["istop"] == 1 for i in warm)
    assert itw.mean() < itc.mean()
    # the oracle's residual of sampled warm solutions, mapped back to coefficients x = R^{-1} y
    x = torch.empty_like(x0)
    B2.from_coords(torch.as_tensor(yw).cuda(), x)
    xh = x.cpu().numpy()
    R = C2.shape[1]
    n = specs2[0].levels[0][0] * specs2[0].K
    for g in (0, 17, 31):
        s = specs2[g]
        Wf, bf = feature_params(s)
        bl = asm.assemble_blocks(s, Wf, bf)
        f = configs.warm_batch_forcing(s, C2[g])
        for j in (0, R - 1):
            h = asm.rhs(s, f[j])
            xj = xh[g * R * n + j * n:g * R * n + (j + 1) * n]
            r = np.linalg.norm(asm.matvec(bl, xj, s.n_rows) - h) / np.linalg.norm(h)
            print(f"group {g} rhs {j}: oracle rel residual {r:.2e}")
            assert r <= btol * (1 + 1e-2)
    B2.destroy()
    W.destroy()
