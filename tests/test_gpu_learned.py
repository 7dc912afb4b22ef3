"""GPU parity of the learned-guess kernels against the FP64 oracle
(oracle/learned.py): perceptron forward, loss gradient and Adam training in
FP32; PCA fit and expansion in FP64."""
import numpy as np
import pytest

from oracle import learned as OL

pytestmark = pytest.mark.gpu


def _net(seed, nin=36, nh=64, nout=24):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, OL.nparams(nin, nh, nout))
    return rng, p, nin, nh, nout


def test_mlp_forward_and_gradient():
    from paper_2403_01007_amd.binding import Mlp
    rng, p, nin, nh, nout = _net(0)
    X = rng.normal(size=(50, nin))
    T = rng.normal(size=(50, nout))
    p32 = p.astype(np.float32).astype(np.float64)  # the device holds FP32 parameters
    net = Mlp(nin, nh, nout, p32)
    Y = net.forward(X).cpu().numpy()
    Yr, _ = OL.forward(p32, X.astype(np.float32).astype(np.float64), nin, nh, nout)
    err = np.abs(Y - Yr).max() / np.abs(Yr).max()
    print(f"[mlp forward] relative error {err:.2e}", flush=True)
    assert err < 2e-5
    loss, g = net.loss_grad(X, T)
    lr_, gr = OL.loss_and_grad(p32, X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64),
                               nin, nh, nout)
    gerr = np.abs(g.cpu().numpy() - gr).max() / np.abs(gr).max()
    print(f"[mlp gradient] loss {loss:.6e} vs {lr_:.6e}, gradient relative error {gerr:.2e}", flush=True)
    assert abs(loss - lr_) < 1e-5 * lr_
    assert gerr < 1e-4


def test_mlp_training_follows_the_oracle():
    from paper_2403_01007_amd.binding import Mlp
    rng, p, nin, nh, nout = _net(1, nin=6, nh=32, nout=5)
    X = rng.normal(size=(64, nin))
    T = np.stack([np.sin(X[:, k % nin]) * np.cos(X[:, (k + 1) % nin]) for k in range(nout)], axis=1)
    order = np.stack([rng.permutation(64)[:16] for _ in range(40)])
    lr = 1e-3
    p32 = p.astype(np.float32).astype(np.float64)
    net = Mlp(nin, nh, nout, p32)
    losses = net.train(X, T, order, lr=lr)
    pr, lr_ref = OL.train(p32, X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64),
                          nin, nh, nout, list(order), 16, lr=lr)
    lerr = np.abs(losses - lr_ref).max() / lr_ref.max()
    perr = np.abs(net.params.cpu().numpy() - pr).max()
    print(f"[mlp training] loss relative error {lerr:.2e}, max parameter difference {perr:.2e}", flush=True)
    assert lerr < 1e-4
    # every Adam step moves a parameter by at most about lr
    assert perr < 0.05 * lr * len(order)
    assert losses[-5:].mean() < losses[:5].mean()


def test_pca_fit_and_expand():
    import torch
    from paper_2403_01007_amd.binding import pca_expand, pca_fit
    rng = np.random.default_rng(2)
    n, d, k = 40, 3000, 8
    # decaying spectrum: well separated leading components
    Q, _ = np.linalg.qr(rng.normal(size=(d, 12)))
    X = rng.normal(size=(n, 12)) * (2.0 ** -np.arange(12)) @ Q.T + rng.normal(size=d)
    m, U, C, w = pca_fit(torch.as_tensor(X, device="cuda:0"), k)
    mr, Ur, Cr, wr = OL.pca_fit(X, k)
    print("[pca] eigenvalue relative error", np.abs(np.array(w) - wr).max() / wr.max(), flush=True)
    assert np.abs(m.cpu().numpy() - mr).max() < 1e-12
    assert np.abs(np.array(w) - wr).max() < 1e-10 * wr.max()
    assert np.abs(U.cpu().numpy() - Ur).max() < 1e-8
    assert np.abs(C.cpu().numpy() - Cr).max() < 1e-8 * np.abs(Cr).max()
    R = pca_expand(m, U, C).cpu().numpy()
    assert np.abs(R - (mr + Cr @ Ur)).max() < 1e-8


def test_learned_guess_gains_and_keeps_results():
    """Train on solved geometries of the trajectory family (o4v12 size, 36
    coordinates): PCA bases of the amplitudes, of the right vectors and of the
    multipliers of every gradient / coupling target, and the perceptron on
    the standardised coefficients.  Held-out geometries are solved twice,
    each sequence in a context of its own: from the plain start and from the
    predicted start.  The predicted start reaches the energies, gradients
    and couplings of the plain start, never falls back in the ground and
    excited solves, and takes fewer iterations in total.  The multiplier
    guess (used or, when its residual is above that of the zero start,
    dropped) never costs iterations: a Krylov solve gains only the
    logarithm of the guess error, about one step per decade, so a guess
    10 % off saves about one step."""
    import torch
    from paper_2403_01007_amd import Context
    from paper_2403_01007_amd.binding import FIELD_R, FIELD_T, Mlp, pca_expand, pca_fit
    from synth_inputs import family_geometries, make_system
    S = make_system("o4v12x36")
    print("[learned guess o4v12x36]", flush=True)
    ns, npair = S.nstates, S.nstates * (S.nstates - 1) // 2
    states, pairs = list(range(ns)), list(S.nacs)
    nt = len(states) + len(pairs)
    mk = lambda: Context(S.o, S.v, S.nj, ns, tol=1e-10, tol_overlap=1e-11)
    ctx = mk()
    nst = 1 + S.o * S.v * (1 + S.o * S.v)
    nm = ctx.multiplier_length()
    ntr = 48
    Xtr = family_geometries(S.ncoord, range(10000, 10000 + ntr))
    Tm = torch.empty((ntr, nst - 1), dtype=torch.float64, device="cuda:0")
    Rm = torch.empty((ntr, ns * nst), dtype=torch.float64, device="cuda:0")
    Mm = torch.empty((ntr, nt * nm), dtype=torch.float64, device="cuda:0")
    Zm = np.zeros((ntr, npair))
    for i, x in enumerate(Xtr):
        ctx.set_hamiltonian_fixed_basis(*S.at(x))
        _, z, _ = ctx.excited()
        *_, M = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, multipliers=True)
        Tm[i] = ctx.get(FIELD_T)
        for k in range(ns):
            Rm[i, k * nst:(k + 1) * nst] = ctx.get(FIELD_R, k)
        Mm[i] = M.reshape(-1)
        Zm[i] = z
    k = 16
    mt, Ut, Ct, _ = pca_fit(Tm, k)
    mr, Ur, Cr, _ = pca_fit(Rm, k)
    mm, Um, Cm, _ = pca_fit(Mm, k)
    Y = np.concatenate([Ct.cpu().numpy(), Cr.cpu().numpy(), Cm.cpu().numpy(), Zm], axis=1)
    mu, sd = Y.mean(axis=0), Y.std(axis=0) + 1e-12
    rng = np.random.default_rng(7)
    nh, nout = 64, Y.shape[1]
    sizes = [(nh, S.ncoord), (nh,), (nh, nh), (nh,), (nout, nh), (nout,)]
    p0 = np.concatenate([rng.normal(0, 1 / np.sqrt(s[1]), s).ravel() if len(s) == 2 else np.zeros(s) for s in sizes])
    net = Mlp(S.ncoord, nh, nout, p0)
    losses = net.train(Xtr, (Y - mu) / sd, np.stack([rng.permutation(ntr)[:32] for _ in range(1500)]), lr=1e-3)
    assert losses[-50:].mean() < 0.2 * losses[:10].mean()
    mu_d, sd_d = torch.as_tensor(mu, device="cuda:0"), torch.as_tensor(sd, device="cuda:0")
    held = family_geometries(S.ncoord, range(20000, 20008))
    plain_ctx, learned_ctx = mk(), mk()
    tot_plain = tot_learned = 0
    for x in held:
        plain_ctx.set_hamiltonian_fixed_basis(*S.at(x))
        E0, _, i0 = plain_ctx.excited()
        g0, d0, m0 = plain_ctx.gradients_and_couplings(states, pairs, S.dh, S.dL)
        learned_ctx.set_hamiltonian_fixed_basis(*S.at(x))
        y = net.forward(x[None, :]).to(torch.float64) * sd_d + mu_d
        _, ig = learned_ctx.ground(pca_expand(mt, Ut, y[:, :k])[0])
        E1, _, i1 = learned_ctx.excited(torch.cat([pca_expand(mr, Ur, y[:, k:2 * k])[0], y[0, 3 * k:]]))
        Mg = pca_expand(mm, Um, y[:, 2 * k:3 * k])[0].reshape(nt, nm)
        g1, d1, m1 = learned_ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, guess=Mg)
        print(f"  iterations plain {i0.iterations} + {m0.iterations}, learned {ig.iterations} + {i1.iterations} + "
              f"{m1.iterations} (multiplier guess {'rejected' if m1.fallback_used else 'used'})", flush=True)
        assert np.abs(E1 - E0).max() < 1e-9
        assert np.abs(g1 - g0).max() < 1e-8 and np.abs(d1 - d0).max() < 1e-8
        assert ig.fallback_used == 0 and i1.fallback_used == 0
        # the two sequences' converged states differ at the solver tolerance,
        # which can move a count by one
        assert m1.iterations <= m0.iterations + 1
        tot_plain += i0.iterations + m0.iterations
        tot_learned += ig.iterations + i1.iterations + m1.iterations
    print(f"  total iterations plain {tot_plain}, learned {tot_learned}", flush=True)
    assert tot_learned < tot_plain
