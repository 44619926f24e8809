"""Learned-closure training on the GPU against the FP64 oracle.

* Gradients: the GPU evaluates forward and backward passes with BF16 operands
  (inputs, activations and the layer-2 gradient rounded to 8 bits) and FP32
  accumulation; the oracle differentiates the same BF16-rounded weights in
  FP64 on unrounded inputs.  Bound: normwise 2e-2 per parameter group.
* Training samples: GPU (FP32 arithmetic) vs the NumPy FP64 oracle of the
  filter/strain/target/feature pipeline, both fed by an FP64 fine run
  (oracle LBM vs GPU FP64 storage, which agree to 1e-12).
"""
import numpy as np
import pytest

from oracle import closure_ref, ref
from paper_2206_15454_amd import closure, inputs
from tests.gpu_common import make_pair, normwise, require_gpu

pytestmark = pytest.mark.gpu

GROUPS = {"W1": slice(0, 576), "b1": slice(576, 640), "W2": slice(640, 4736),
          "b2": slice(4736, 4800), "w3": slice(4800, 4864), "b3": slice(4864, 4865)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return closure.join(rng.normal(size=(64, 9)) / 3.0 * scale, rng.normal(size=64) * 0.1,
                        rng.normal(size=(64, 64)) / 8.0 * scale, rng.normal(size=64) * 0.1,
                        rng.normal(size=64) / 8.0 * scale, -0.5)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    mean = rng.normal(size=9)
    std = rng.uniform(0.5, 2.0, size=9)
    X = (mean + std * rng.normal(size=(n, 9))).astype(np.float32)
    return X, mean, std


def test_gradient_matches_oracle():
    import torch
    from paper_2206_15454_amd import lbm

    n, s = 1000, 2e-4  # a ragged batch (not a multiple of 64)
    X, mean, std = _data(n, 1)
    y = (s * np.random.default_rng(2).uniform(0.1, 3.0, size=n)).astype(np.float32)
    p = _random_params(3)
    tr = lbm.Trainer(p, mean, std, s, max_batch=1024)
    loss_gpu = tr.step(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), update=False)
    _, g_gpu = tr.get()
    pm = closure.stored_params(p)  # weights as the GPU uses them (bf16), biases f32
    Z = (X.astype(np.float64) - np.float32(mean).astype(np.float64)) / np.float32(std).astype(np.float64)
    loss_ref, g_ref = ref.mlp_loss_grad(pm, Z, y.astype(np.float64) / np.float64(np.float32(s)))
    print("loss gpu", loss_gpu, "oracle", loss_ref)
    assert loss_gpu == pytest.approx(loss_ref, rel=1e-2)
    for name, sl in GROUPS.items():
        e = normwise(g_gpu[sl].astype(np.float64), g_ref[sl])
        print(f"grad {name}: normwise {e:.3e}")
        assert e <= 2e-2, name
    tr.close()


def test_training_fits_a_teacher_network():
    """Targets from a random teacher network; the student (another random
    init) is trained with Adam on the GPU: the loss falls by more than 10x, and
    the GPU-reported loss agrees with the oracle's loss of the trained
    parameters."""
    import torch
    from paper_2206_15454_amd import lbm

    n, s = 16384, 1e-4
    X, mean, std = _data(n, 4)
    Z = (X.astype(np.float64) - mean) / std
    teacher = closure.stored_params(_random_params(5, scale=0.7))
    y = (s * np.log1p(np.exp(ref.mlp_apply(teacher, Z)))).astype(np.float32)
    tr = lbm.Trainer(_random_params(6), mean, std, s, lr=3e-3, max_batch=4096)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    first = None
    for it in range(400):
        b = (it % 4) * 4096
        l = tr.step(Xd[b:b + 4096], yd[b:b + 4096], update=True, loss=(it % 50 == 0))
        if first is None:
            first = l
    p, _ = tr.get()
    Zf = (X.astype(np.float64) - np.float32(mean).astype(np.float64)) / np.float32(std).astype(np.float64)
    final_ref, _ = ref.mlp_loss_grad(closure.stored_params(p), Zf,
                                     y.astype(np.float64) / np.float64(np.float32(s)))
    final_gpu = tr.step(Xd[:4096], yd[:4096], update=False)
    print("loss first", first, "final gpu", final_gpu, "final oracle (all data)", final_ref)
    assert final_ref < first / 10
    assert final_gpu == pytest.approx(
        ref.mlp_loss_grad(closure.stored_params(p), Zf[:4096],
                          y[:4096].astype(np.float64) / np.float64(np.float32(s)))[0], rel=5e-2)
    tr.close()


def test_closure_samples_match_oracle():
    w = inputs.scaled(inputs.C1, 32, 16, 12, noise=0.3)
    o, g = make_pair(w, storage="f64", seed=11)
    o.step(12)
    g.step(12)
    _, uo, no, _ = o.moments()
    lad_c = np.linspace(0.3, 0.0, w.ny // 2)
    Xo, yo, _ = closure_ref.samples(uo, no, 0.52, 4.0, lad_c)
    Xg, yg = g.closure_samples(0.52, 4.0, lad_c)
    Xg = Xg.cpu().numpy().astype(np.float64)
    yg = yg.cpu().numpy().astype(np.float64)
    ey = normwise(yg, yo)
    print("samples: target normwise", ey, "max target", yo.max(), "nonzero", (yo > 0).mean())
    assert yo.max() > 0 and ey <= 5e-3
    # each feature's error relative to the natural scale of its column: the
    # trace of P (x0) and tr P^3 (x2) nearly cancel in a near-incompressible
    # flow, so they are measured against |P| = x5 and |P|^3
    P = np.max(np.abs(Xo[:, 5]))
    scale = [P, P * P, P ** 3, P, P * P, P] + [np.max(np.abs(Xo[:, c])) for c in (6, 7, 8)]
    for c in range(9):
        ec = float(np.max(np.abs(Xg[:, c] - Xo[:, c])) / scale[c])
        print(f"feature {c}: error / scale {ec:.3e}")
        assert ec <= 2e-3, c


def test_trained_closure_beats_smagorinsky_a_priori():
    """What the trained network gains over the method without it, a priori:
    filtered samples of a fresh run at twice the resolution (the canopy
    case's physics on 256x128x128, so 128x64x64 coarse samples after 20 000
    fine steps) are predicted by the committed network and by the Smagorinsky
    closure of the coarse case (Sec. 2.2, in the form of the step, from the
    same feature |P|).  The network's loss must be a small fraction of the
    Smagorinsky loss; on 16.8 M samples of the full-size case the ratio is
    0.008."""
    import math

    import torch

    from paper_2206_15454_amd import lbm, studies

    wf = inputs.scaled(inputs.C4, 256, 128, 128)
    wc = inputs.scaled(inputs.C2, 128, 64, 64)
    rho, u = inputs.init_fields_torch(wf, torch.device("cuda"))
    fine = studies.make(wf, "f32", rho, u)
    fine.step(20000)
    X, y = fine.closure_samples(wc.tau0, wc.lad_lalic[0], studies._lad(wc))
    d = fine.diag()
    fine.close()
    assert d["nonfinite"] == 0
    p, mean, std, lo, hi, s, _ = closure.read_blob(closure.trained_blob())
    batch = 8192
    n = (y.numel() // batch) * batch
    var = float((y[:n].double() / s).var())
    assert var > 1e-3, var  # the flow has subfilter stress to predict
    tr = lbm.Trainer(p, mean, std, s, max_batch=batch)
    l_net = sum(tr.step(X[b:b + batch], y[b:b + batch], update=False)
                for b in range(0, n, batch)) * batch / n
    tr.close()
    xs = 6.0 * math.sqrt(2.0) * wc.c_smag * X[:n, 5].double()
    nu_s = xs / (6.0 * (torch.sqrt(wc.tau0 * wc.tau0 + xs) + wc.tau0))
    l_smag = float(((nu_s - y[:n].double()) / s).pow(2).mean())
    print(f"a priori on {n} samples: target variance {var:.3f}, network loss {l_net:.4f} "
          f"(explained {1 - l_net / var:.3f}), Smagorinsky loss {l_smag:.4f} "
          f"(explained {1 - l_smag / var:.3f})")
    assert l_net < 0.25 * l_smag
    assert 1.0 - l_net / var > 0.5
