"""The differentiation case at full size: 100k Gaussians (clustered-scene distributions, SH1), 8 views
at 800x800 of random (camera, t), and the L2 loss against a target: the same scene with
N(0, 0.01) noise on every raw parameter, rendered by the oracle.

L = mean over the 3 x 800 x 800 values of (image - target)^2, so dL/dimage =
2 (image - target) / (3 H W).  Both sides differentiate with that upstream gradient, taken
from the oracle's image (zero at pixels the oracle flags as near a threshold); the
parameter gradients of the 8 views are accumulated into one set and compared per group
at the 1e-3 relative bar.  The oracle's adjoint is itself pinned to finite differences
(test_oracle_pins)."""
import numpy as np
import pytest

import oracle
from _helpers import compare_images
from paper_2503_22159_amd import inputs
from test_gpu_backward import GROUPS, compare_group

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_22159_amd import render

    return render


@pytest.mark.timeout(400)
def test_fit_case_l2_loss_gradients(R):
    import torch

    sc, views, target_scene = inputs.fit_case()
    ds = R.DeviceScene.from_inputs(sc)
    grads = R.grads_like(ds)
    gsum = None
    loss = 0.0
    for i, (cam, t) in enumerate(views):
        target = oracle.render(target_scene, cam, t)[2]["img"]
        img, st = R.render_forward(ds, cam, t, (0.0, 0.0, 0.0))
        proj, bins, res = oracle.render(sc, cam, t)
        stats = compare_images(img.cpu().numpy(), st.final_T.cpu().numpy(),
                               st.n_contrib.cpu().numpy().view(np.uint32), res)
        diff = res["img"] - target
        loss += float((diff * diff).mean()) / len(views)
        dL = (2.0 / diff.size) * diff * ~(res["flags"] > 0)[None]
        R.render_backward(ds, cam, t, (0.0, 0.0, 0.0), st, torch.from_numpy(dL.astype(np.float32)).cuda(), grads)
        gp, _, _ = oracle.render_grad(sc, cam, t, dL)
        gsum = gp if gsum is None else {k: gsum[k] + gp[k] for k in gsum}
        print("fit_case view", i, "instances", bins["I"], stats)
    torch.cuda.synchronize()
    gg = {k: grads[k].cpu().numpy().astype(np.float64) for k in GROUPS}
    errs = {k: compare_group(k, gg[k], gsum[k]) for k in GROUPS}
    print("fit_case loss", loss, "grad rel err", errs)
    assert loss > 0.0
