"""Driver of the learned preconditioner: harvest training pairs from the
solver's own Jacobi-PCG runs and train the network, through the C ABI.

Every arithmetic step runs in libmffv (residuals, scaling, network forward and
backward, Adam); this module only orders the calls and keeps the tensors.

Everything happens in the Jacobi-scaled space A~ = D^-1/2 A D^-1/2. For a
scaled residual r_hat the ideal output is the error A~^-1 r_hat; the network is
trained so that z = r_hat + N(r_hat, feature) minimises the energy functional
z' A~ z - 2 z' r_hat, whose minimiser is that error, so a residual alone is a
training example and no reference solve is needed (with a known error target
the same loss is the energy norm of the prediction error). With N = 0 the
preconditioner is Jacobi.

Training inputs. Residuals of Jacobi-PCG iterates (``harvest``) concentrate on
the smooth error modes that a 9x9x9 receptive field cannot invert, and a
network trained on them alone amplifies smooth components and makes flexible
CG diverge. The recipe used here (``train_preconditioner``) therefore trains
on white-noise residuals over the held-in operators and then adds residuals
from the solver's own flexible-CG runs with the current network (``dagger``);
harvested Jacobi pairs remain available as a validation set (their energy
loss is reported by ``evaluate_loss``).
"""
from __future__ import annotations

import random
from dataclasses import dataclass

import torch

from . import mffv

DEFAULT_ITERS = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)


@dataclass
class Sample:
    grid: mffv.Grid          # the system's operator (kept alive with the pair)
    r_hat: torch.Tensor
    target: torch.Tensor
    iteration: int


def reference_solution(grid: mffv.Grid, b: torch.Tensor, tol: float = 1e-10) -> torch.Tensor:
    x = torch.zeros(grid.n, dtype=torch.float64, device=b.device)
    st, info = mffv.cg_solve_f64(grid, b.double(), x,
                                 mffv.default_opts(tol=tol, precision=mffv.FP32_IR,
                                                   precond=mffv.PRECOND_JACOBI))
    if st != mffv.OK:
        raise RuntimeError(f"reference solve failed: {info}")
    return x


def harvest(grid: mffv.Grid, b: torch.Tensor, iters=DEFAULT_ITERS, x_star=None) -> list:
    """Training pairs at the given Jacobi-PCG iteration counts of one system."""
    if x_star is None:
        x_star = reference_solution(grid, b)
    out = []
    x = torch.zeros(grid.n, dtype=torch.float32, device=b.device)
    for k in iters:
        x.zero_()
        st, info = mffv.cg_solve(grid, b, x, mffv.default_opts(
            tol=1e-12, max_iter=k, precond=mffv.PRECOND_JACOBI))
        if info["iters"] < k:       # converged before k: no more distinct pairs
            break
        r_hat, target = (torch.empty(grid.n, dtype=torch.float32, device=b.device)
                         for _ in range(2))
        mffv.harvest_pair(grid, b, x, x_star, r_hat, target)
        out.append(Sample(grid, r_hat, target, k))
    return out


def white_residuals(shape, count: int, seed: int):
    """``count`` independent standard-normal FP32 fields of the grid's shape
    (NumPy PCG64 from ``seed``), each rescaled to unit RMS."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = rng.standard_normal((count,) + tuple(shape)).astype(np.float32)
    out /= np.sqrt(np.mean(out.reshape(count, -1) ** 2, axis=1)).reshape((count,) + (1,) * len(shape))
    return out


def white_samples(systems, count: int, seed: int) -> list:
    """``count`` white-noise residual samples spread over the systems' operators."""
    out = []
    per = -(-count // len(systems))
    for i, (grid, _b) in enumerate(systems):
        fields = white_residuals(grid.shape, per, seed + i)
        for f in fields:
            if len(out) == count:
                break
            out.append(Sample(grid, torch.from_numpy(f.ravel()).cuda(), None, -1))
    return out


def dagger(net: mffv.Net, systems, iters=(2, 8, 32, 64, 128)) -> list:
    """Residual samples from the solver's own flexible-CG runs with ``net``."""
    out = []
    for grid, b in systems:
        x = torch.zeros(grid.n, dtype=torch.float32, device=b.device)
        for k in iters:
            x.zero_()
            st, info = mffv.cg_solve(grid, b, x, mffv.default_opts(
                tol=1e-12, max_iter=k, precond=mffv.PRECOND_LEARNED, net=net))
            if info["iters"] < k:
                break
            r_hat, target = (torch.empty(grid.n, dtype=torch.float32, device=b.device)
                             for _ in range(2))
            mffv.harvest_pair(grid, b, x, x.double(), r_hat, target)
            out.append(Sample(grid, r_hat, None, k))
    return out


def smoothed(samples: list, omega: float) -> list:
    """The samples as the network sees them between the Jacobi sweeps of the
    solver's preconditioner: r_hat -> (I - omega A~) r_hat on each sample's
    operator (mffv_nn_smooth_sample); samples with a target are kept as they are."""
    if omega <= 0:
        return samples
    out = []
    for s in samples:
        if s.target is not None:
            out.append(s)
            continue
        r1 = torch.empty_like(s.r_hat)
        mffv.nn_smooth_sample(s.grid, omega, s.r_hat, r1)
        out.append(Sample(s.grid, r1, None, s.iteration))
    return out


LAYERS = ((2, 16), (16, 16), (16, 16), (16, 1))


def init_params(seed: int = 0):
    """He-normal weights with the last layer zero (the network starts as
    Jacobi), zero biases; the library's parameter layout (W[27][cin][cout], b)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(LAYERS):
        W = rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=27 * ci * co)
        if li == len(LAYERS) - 1:
            W[:] = 0.0
        parts += [W, np.zeros(co)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == mffv.net_num_params()
    return p


def fcg_iterations(net: mffv.Net, systems, max_iter=20000, omega: float | None = None) -> int:
    """Total flexible-CG iterations to 1e-6 over the systems (validation metric);
    a system that does not converge within max_iter (a number, or one per
    system) counts max_iter. omega: the weight of the Jacobi sweeps around the
    network (None: the library's default)."""
    caps = max_iter if isinstance(max_iter, (list, tuple)) else [max_iter] * len(systems)
    kw = {} if omega is None else {"nn_smooth": float(omega)}
    tot = 0
    for (grid, b), cap in zip(systems, caps):
        x = torch.zeros(grid.n, dtype=torch.float32, device=b.device)
        st, info = mffv.cg_solve(grid, b, x, mffv.default_opts(
            precond=mffv.PRECOND_LEARNED, net=net, max_iter=int(cap), **kw))
        tot += info["iters"] if st == mffv.OK else int(cap)
    return tot


def select_smoothing(net: mffv.Net, systems, omegas=(0.5, 0.7, 0.85, 0.95, 1.0, 1.1)):
    """The sweep weight omega (opts.nn_smooth) for a trained network: the one
    with the fewest flexible-CG iterations on the given (held-in) systems; the
    first of equal counts. Returns (omega, {omega: iterations})."""
    scores = {float(w): fcg_iterations(net, systems, omega=w) for w in omegas}
    best = min(scores, key=lambda w: (scores[w], list(scores).index(w)))
    return best, scores


def train_preconditioner(systems, validation=None, n_white: int = 256, epochs: int = 24,
                         lr: float = 2e-3, lr_final: float = 1e-4, dagger_rounds: int = 2,
                         dagger_epochs: int = 6, seed: int = 0, relu: bool = True,
                         loss: int = 0, init=None, smooth: float = 0.0, log=None) -> mffv.Net:
    """The training recipe on held-in systems [(grid, b), ...].

    White-noise residuals with the energy functional, then ``dagger_rounds``
    rounds that add residuals of the solver's own flexible-CG runs with the
    current network. After every epoch the network is scored by the total
    flexible-CG iteration count on the validation systems (default: the first
    two held-in systems) and the best parameters so far are kept; the zero
    network (Jacobi) is the first candidate, so the result is never worse
    than Jacobi on the validation systems. With ``init`` (a parameter vector,
    e.g. a network trained on another field) training continues from it
    (fine-tuning), and that network is the first candidate instead. With
    ``smooth`` = omega > 0 every target-free sample is first passed through
    the first Jacobi sweep (:func:`smoothed`), so that the network is trained
    on the residuals it sees inside the solver's preconditioner.
    """
    import numpy as np
    validation = systems[:2] if validation is None else validation
    p0 = init_params(seed) if init is None else np.array(init, dtype=np.float32).ravel()
    net = mffv.net_create(p0)
    mffv.net_set_activation(net, relu)
    mffv.net_set_loss(net, loss)
    best_p = p0.copy()                      # the starting network (zero last layer: Jacobi)
    caps = []
    for sysv in validation:                 # a candidate may take twice the start's count at most
        caps.append(2 * fcg_iterations(net, [sysv]) + 10)
    best = sum((c - 10) // 2 for c in caps)
    if log:
        log(f"validation FCG iterations with the {'zero' if init is None else 'starting'} network: {best}")

    def run(samples, n_ep, lr0, lr1, tag, sd):
        nonlocal best, best_p
        rng = random.Random(sd)
        order = list(range(len(samples)))
        total, step = n_ep * len(samples), 0
        for ep in range(n_ep):
            rng.shuffle(order)
            for i in order:
                s = samples[i]
                cur = lr0 * (lr1 / lr0) ** (step / max(1, total - 1))
                mffv.nn_train_step(net, s.grid, s.r_hat, s.target, cur)
                step += 1
            it = fcg_iterations(net, validation, caps)
            if it < best:
                best = it
                best_p, _ = mffv.net_get_params(net)
            if log:
                log(f"{tag} epoch {ep}: validation FCG iterations {it} (best {best})")

    run(smoothed(white_samples(systems, n_white, seed), smooth), epochs, lr, lr_final, "white", seed)
    for r in range(dagger_rounds):
        mffv.net_set_params(net, best_p)
        extra = dagger(net, systems)
        more = white_samples(systems, n_white // 2, seed + 1000 * (r + 1))
        run(smoothed(extra + more, smooth), dagger_epochs, lr / 4, lr_final, f"dagger{r}", seed + r + 1)
    mffv.net_set_params(net, best_p)
    del np
    return net


def train_best_of(systems, select_on, seeds=(0, 1, 2), log=None, **kw):
    """Train one network per seed with :func:`train_preconditioner` and keep
    the one with the fewest flexible-CG iterations on the ``select_on``
    systems (held-in systems at the size the network will be used at: the
    recipe's epoch selection works on small systems, and a network's benefit
    at full size varies between seeds). Returns (network, {seed: iterations})."""
    best, best_it, scores = None, None, {}
    for seed in seeds:
        net = train_preconditioner(systems, seed=seed, log=log, **kw)
        it = fcg_iterations(net, select_on)
        scores[seed] = it
        if log:
            log(f"seed {seed}: flexible-CG iterations on the selection systems {it}")
        if best_it is None or it < best_it:
            if best is not None:
                best.close()
            best, best_it = net, it
        else:
            net.close()
    return best, scores


def train(net: mffv.Net, samples: list, epochs: int = 4, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, lr_final: float | None = None):
    """Adam over the samples in shuffled order; returns the per-epoch mean loss
    (samples with target None use the energy functional)."""
    rng = random.Random(seed)
    order = list(range(len(samples)))
    hist = []
    step, total = 0, epochs * len(samples)
    for ep in range(epochs):
        rng.shuffle(order)
        losses = []
        for i in order:
            s = samples[i]
            frac = step / max(1, total - 1)
            cur = lr if lr_final is None else lr * (lr_final / lr) ** frac
            loss = mffv.nn_train_step(net, s.grid, s.r_hat, s.target, cur, want_loss=True)
            losses.append(loss)
            step += 1
            if log_every and step % log_every == 0:
                print(f"[train] step {step}/{total} loss {loss:.4f}", flush=True)
        hist.append(sum(losses) / len(losses))
    return hist


def evaluate_loss(net: mffv.Net, samples: list) -> float:
    tot = 0.0
    for s in samples:
        tot += mffv.nn_loss_grad(net, s.grid, s.r_hat, s.target)
    return tot / max(1, len(samples))
