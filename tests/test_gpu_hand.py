"""The hand-derived anisotropic kernels (second GPU parity source and speed
reference) against the oracle, and the compiled kernels against them."""
import numpy as np
import pytest

from paper_2508_15967_amd import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _hand_run(w, ckpt=100):
    torch = U.torch_mod()
    from paper_2508_15967_amd import hand
    hm = hand.medium_struct(w.medium)
    x0, k0, om, s = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega), U.dev(w.medium.scales)
    xo, ko = torch.empty_like(x0), torch.empty_like(k0)
    nc = (w.n_steps + ckpt - 1) // ckpt
    cp = torch.empty((nc, 7, w.n), dtype=torch.float64, device="cuda")
    hand.trace(hm, x0, k0, om, s, w.dt, w.n_steps, xo, ko, ckpt, cp)
    lx = (2.0 * (xo - U.dev(w.targets))).contiguous()
    gx0, gk0, gs = torch.empty_like(x0), torch.empty_like(k0), torch.empty_like(s)
    hand.adjoint(hm, om, s, w.dt, w.n_steps, ckpt, cp, lx, None, gx0, gk0, gs)
    torch.cuda.synchronize()
    return {"x": xo.cpu().numpy(), "k": ko.cpu().numpy(), "gx0": gx0.cpu().numpy(),
            "gk0": gk0.cpu().numpy(), "gs": gs.cpu().numpy()}


def test_hand_matches_oracle(oracle):
    w = W.make("5", 512)
    w.n_steps = 1000
    h = _hand_run(w)
    bad, o = U.ill_conditioned(oracle, w)
    ex, ek = U.ray_errors(h, o, w.omega, w.dim)
    assert ex[~bad].max() < U.TOL and ek[~bad].max() < U.TOL
    lam = np.concatenate([2 * (o["x"] - w.targets), np.zeros_like(o["k"])])
    lam0, go = oracle.adjoint(w, lam)
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(h["gk0"], lam0[3:]) < 1e-9 and rel(h["gx0"], lam0[:3]) < 1e-9
    assert rel(h["gs"], go) < 1e-9


def test_compiled_matches_hand():
    """Graph-generated forward and adjoint against the hand-derived kernels on
    16,384 rays x 2,000 steps of workload 5."""
    from tests.test_gpu_adjoint import _gpu_grad
    w = W.make("5", 16384)
    w.n_steps = 2000
    h = _hand_run(w)
    g = _gpu_grad(w)
    ex = np.linalg.norm(g["x"] - h["x"], axis=0) / np.maximum(np.linalg.norm(h["x"], axis=0), 1)
    assert np.quantile(ex, 0.99) < 1e-11
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(g["gp"][0], h["gs"]) < 1e-8
    assert np.quantile(np.abs(g["gk0"] - h["gk0"]).max(0) / np.abs(h["gk0"]).max(0), 0.99) < 1e-9
