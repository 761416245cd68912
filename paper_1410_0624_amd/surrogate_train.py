"""Training loop of the learned surrogate (argument marshalling only: every
step runs in the library's kernels through cd_surrogate_train_step).

The targets are the method's own columns: for each training field the caller
builds the tree and runs cd_column_densities (FP32), and the network learns
ln N of random leaves of those fields."""
from __future__ import annotations

import math

import numpy as np

from . import colden


def norms(trees, w: colden.Weights, Ns, sample: int = 65536, seed: int = 0) -> tuple:
    """Input and output normalisation (in_shift, in_scale, out_shift,
    out_scale) from the training data.  Inputs: centred on the mean ln n of
    the training leaves, scaled so that the out-of-box value ln 1e-10 lands
    at -4 (or by the spread of ln n if that is wider).  Outputs: mean and
    spread of the unscaled targets ln(N_ext + 1e17) (computed by the library)
    over a sample of leaves of each training tree."""
    import torch

    dev = Ns[0].device
    probe = colden.Surrogate(w.D, 16, colden.CD_SURR_FP32, 0, norm=(0.0, 1.0, 0.0, 1.0))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    ln_n, ln_e = [], []
    for tree, N in zip(trees, Ns):
        cells = torch.randint(0, tree.n_leaf, (sample,), device=dev, generator=gen, dtype=torch.int64)
        T = torch.empty((sample, w.D), dtype=torch.float32, device=dev)
        probe.targets(tree, w, N, cells, T)
        ln_e.append(T.cpu().numpy().astype(np.float64).ravel())
        leaf = tree._keep_leaf[cells].cpu().numpy().astype(np.float64)
        ln_n.append(np.log(np.maximum(leaf, 1e-10)))
    probe.close()
    ln_n, ln_e = np.concatenate(ln_n), np.concatenate(ln_e)
    mu = float(ln_n.mean())
    sc = max(float(ln_n.std()), (mu - np.log(1e-10)) / 4.0)
    return (mu, sc, float(ln_e.mean()), float(max(ln_e.std(), 1e-3)))


def fit(surr: colden.Surrogate, trees, w: colden.Weights, Ns, steps: int, batch: int = 4096, lr: float = 2e-3,
        lr_final: float = 1e-4, seed: int = 0, log_every: int = 0):
    """`steps` Adam steps, cycling over the training trees, each on `batch`
    random leaves; learning rate decays geometrically from lr to lr_final.
    Returns the logged (step, loss) pairs."""
    import torch

    dev = Ns[0].device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    log = []
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    for k in range(steps):
        i = k % len(trees)
        cells = torch.randint(0, trees[i].n_leaf, (batch,), device=dev, generator=gen, dtype=torch.int64)
        want = log_every > 0 and (k % log_every == 0 or k == steps - 1)
        loss = surr.train_step(trees[i], w, Ns[i], cells, lr * decay ** k, want_loss=want)
        if want:
            if not math.isfinite(loss):
                raise FloatingPointError(f"surrogate loss {loss} at step {k}")
            log.append((k, loss))
    return log
