"""Differentiation form: the correlator and the receive model behind
torch.autograd.Function, checked by finite differences (FP64 gradcheck) and
against the oracle's adjoint and loss gradient."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, frames, host, perr

pytestmark = pytest.mark.gpu


def _plan(N, T, L, R):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R)


def test_gradcheck_fp64_tiny_instance():
    """FP64 gradcheck (finite differences) on N=31, T=2, L=4, R=2."""
    from paper_2206_05506_amd.autograd import PnceCorrelate, PnceSynthesize
    cfg = synth.GRADCHECK
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        Y = dev(synth.gaussian((1, cfg.R, cfg.N), 1), torch.complex128).requires_grad_(True)
        X = dev(synth.gaussian((1, cfg.R, cfg.K), 2), torch.complex128).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda y: PnceCorrelate.apply(y, p, "f64"), (Y,),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)
        assert torch.autograd.gradcheck(lambda x: PnceSynthesize.apply(x, p, "f64"), (X,),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.mark.parametrize("prec", ["f32", "f32s", "exact", "exact32"])
def test_backward_equals_oracle_adjoint(prec):
    from paper_2206_05506_amd.autograd import correlate
    N, T, L, R, B = 255, 4, 16, 8, 3
    Y = synth.gaussian((B, R, N), 3).astype(np.complex64)
    G = synth.gaussian((B, R, T * L), 4).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        Yd = dev(Y).requires_grad_(True)
        H = correlate(Yd, p, prec)
        (gY,) = torch.autograd.grad(H, Yd, grad_outputs=dev(G))
        s = p.sequence()
    assert perr(host(gY), oracle.adjoint(G, s)) <= 1e-5


@pytest.mark.parametrize("prec", ["f32s", "exact", "exact32"])
def test_loss_gradient_equals_oracle(prec):
    from paper_2206_05506_amd.autograd import residual_loss
    N, T, L, R, B = 127, 4, 16, 6, 2
    y = synth.gaussian((B, R, N), 5).astype(np.complex64)
    x = synth.gaussian((B, R, T * L), 6).astype(np.complex64) * 0.1
    with _plan(N, T, L, R) as p:
        xd = dev(x).requires_grad_(True)
        loss = residual_loss(dev(y), xd, p, prec)
        (g,) = torch.autograd.grad(loss, xd)
        s = p.sequence()
    ref_loss, ref_g = oracle.loss_grad(y, s, x)
    assert abs(float(loss.detach()) - ref_loss) <= 1e-5 * ref_loss
    assert perr(host(g), ref_g) <= 1e-5


def _per_frame_loss(y, x, p):
    from paper_2206_05506_amd.autograd import synthesize
    r = y - synthesize(x, p, "f32s")
    return (r.real ** 2 + r.imag ** 2).sum(dim=(1, 2))


def test_differentiation_workload_refinement_trajectory():
    """Differentiation workload (N=1023, T=16, L=64 -> T*L = 1024 > N, R=128,
    1024 frames, complex64): 5 refinement steps as gradient descent on
    ||y - P x||^2 through autograd. Every iterate matches the oracle's FP64
    iterate with the same step count on sampled frames, and so does each
    sampled frame's loss trajectory; so does the library's own five-step
    refinement of the whole batch."""
    from paper_2206_05506_amd.autograd import refine_by_gradient
    cfg = synth.DIFF
    pick = [0, 511, 1023]
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        assert p.lag_alias
        s = p.sequence()
        d = synth.batch_draws(cfg)
        y, _ = oracle.received(s, d["h"], d["w"], d["snr_db"])
        y = y.astype(np.complex64)
        yd = dev(y)
        xs, losses = refine_by_gradient(yd, p, 5, "f32s")
        traj = [host(_per_frame_loss(yd, x, p))[pick] for x in xs]
        got = [host(x[pick]) for x in xs]
        del xs
        X = p.estimate(yd, "f32s")
        p.refine(yd, X, 5)                       # the library's own refinement
        lib5 = host(X[pick])
    its = oracle.refine(y[pick], s, cfg.K, 5)
    err = perr(lib5, its[5])
    print(f"library refinement, 5 steps: relerr {err:.2e}")
    assert err <= 1e-5
    for k in range(6):
        err = perr(got[k], its[k])
        ref_l = [oracle.loss_grad(y[pick][i:i + 1], s, its[k][i:i + 1])[0] for i in range(3)]
        print(f"step {k}: iterate relerr {err:.2e}, loss {traj[k]} vs {ref_l}")
        assert err <= 1e-5
        assert np.allclose(traj[k], ref_l, rtol=1e-5)
    assert len(losses) == 6 and np.all(np.isfinite(losses))


def test_autograd_through_conjugate_views():
    """Inputs and incoming gradients that are lazy conjugate views are
    resolved before the kernels read them."""
    from paper_2206_05506_amd.autograd import correlate
    N, T, L, R, B = 63, 3, 8, 4, 2
    Y = synth.gaussian((B, R, N), 31).astype(np.complex64)
    G = synth.gaussian((B, R, T * L), 32).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        Yd = dev(Y).requires_grad_(True)
        H = correlate(Yd.conj(), p, "f32s")
        (gY,) = torch.autograd.grad(H, Yd, grad_outputs=dev(G).conj())
        s = p.sequence()
        Hh = host(H)
    assert perr(Hh, oracle.correlate(np.conj(Y), s, T * L)) <= 1e-5
    # d/dY of conj(Y) P with incoming conj(G): conj(conj(G) P^T / N) = G P^T / N
    assert perr(host(gY), oracle.adjoint(G, s)) <= 1e-5
