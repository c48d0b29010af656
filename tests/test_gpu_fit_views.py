"""GPU checks of the view-batched fitting loop (a random subset of camera
views per step, as the paper's training samples its supervised points from
randomly selected views): accumulation over views against one backward of
the whole point set, convergence, and resume from a checkpoint."""
import numpy as np
import pytest
import torch

from paper_2512_12459_amd import scenes as S
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

VIEWS, RES = 4, 64


@pytest.fixture(scope="module")
def case():
    from paper_2512_12459_amd import radiance as R
    R.C.lib()   # fail loudly if the library is missing
    gt, x = S.workload("fit200k", views=VIEWS, res=RES)
    start = S.perturb_field(gt, 2)
    xd = torch.from_numpy(x).cuda()
    dev = [torch.from_numpy(a).cuda() for a in gt.arrays()]
    qs = R.QuerySet(xd)
    T = R.eval_radiance(R.Grid(qs).build(*dev), *dev)
    torch.cuda.synchronize()
    return R, start, xd, T


def _fitter(case, k, seed=0):
    from paper_2512_12459_amd.fit import Field, ViewBatchFitter
    R, start, xd, T = case
    return ViewBatchFitter(Field(*start.arrays()), xd, T, [RES * RES] * VIEWS, k, seed=seed)


def test_all_views_accumulate_like_one_backward_of_all_points(case):
    R, start, xd, T = case
    say("case: view-batched accumulation, 4 views of 64x64, 200k Gaussians")
    fit = _fitter(case, VIEWS)
    fit.accumulate(views=list(range(VIEWS)))
    torch.cuda.synchronize()
    g_views = {k: v.cpu().numpy().astype(np.float64) for k, v in fit.f.g.items()}
    loss_views = fit.loss.item()
    # one grid over every point; each point's upstream gradient 2 (L - T) / q_view
    dev = list(fit.f.arrays())
    grid = R.Grid(R.QuerySet(xd)).build(*dev)
    L = R.eval_radiance(grid, *dev)
    d = (L - T).cpu().numpy()
    dL = (np.float32(2.0 / (RES * RES)) * d).astype(np.float32)
    g_all = R.eval_radiance_backward(grid, *dev, torch.from_numpy(dL).cuda())
    torch.cuda.synchronize()
    want = float(np.sum(d.astype(np.float64) ** 2))
    assert abs(loss_views - want) <= 1e-5 * want, (loss_views, want)
    for k, v in g_all.items():
        ref = v.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(g_views[k] - ref) / np.linalg.norm(ref)
        say(f"  {k}: relative 2-norm difference {err:.2e}")
        assert err <= 1e-4, k


def test_view_batches_fit_and_resume(case, tmp_path):
    say("case: view-batched fitting, one view per step, checkpoint after 15 steps")
    fit = _fitter(case, 1, seed=5)
    p0 = fit.current_psnr()
    drawn = []
    for _ in range(15):
        fit.step()
        drawn += fit.last_views
    ck = str(tmp_path / "views.npz")
    fit.save(ck)
    rest = []
    for _ in range(25):
        fit.step()
        rest += fit.last_views
    p1 = fit.current_psnr()
    say(f"  PSNR {p0:.2f} -> {p1:.2f} dB over 40 steps; views drawn {sorted(set(drawn + rest))}")
    assert np.isfinite(p1) and p1 > p0 + 3.0
    assert len(set(drawn + rest)) == VIEWS
    again = _fitter(case, 1, seed=99).load(ck)
    again_views = []
    for _ in range(25):
        again.step()
        again_views += again.last_views
    assert again_views == rest          # the generator's state came back
    assert again.t == fit.t
    assert abs(again.current_psnr() - p1) <= 0.05
