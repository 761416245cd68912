"""Training of the learned surrogate (argument marshalling only: every step
runs in the library's kernels).

A network serves one leaf level L (8 or 9).  Its labels are the method's own
near-shell columns (dl = 1..3) on grids of that level: for each training
field the tree at level L is built and the table of per-row targets
(cd_surrogate_row_targets: one row per level-7 cell, a block of D per oct
inside it) is kept.  A 2^8 training field serves a network of L = 9 through
its refinement into 2^9 equal leaves: the external shells of a 2^9 oct read
pyramid levels 0 .. 8 only, and those are the 2^8 field itself, which also
supplies the features."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import colden, synth


@dataclass
class LabelledField:
    tree: colden.Tree  # features (pyramid levels 0 .. 8)
    leaf: object       # the tree's leaf tensor (kept alive)
    T_rows: object     # [2^21, Dout] unscaled row targets
    ln_n: np.ndarray   # ln n of sampled leaves (input normalisation)


def label_field(tin, w: colden.Weights, leaf_level: int, device, ln_sample: int = 65536,
                seed: int = 0) -> LabelledField:
    """Tree of a uniform field `tin` (2^8 or 2^leaf_level) for the features
    and the method's row targets at `leaf_level`."""
    import torch

    leaf = torch.from_numpy(tin.leaf_n).to(device)
    tree = colden.Tree(tin, leaf, max_dirs=w.D)
    if tin.max_level == leaf_level:
        tl, ll = tree, leaf
    elif tin.max_level + 1 == leaf_level:
        fine = synth.refine_uniform(tin)
        ll = torch.from_numpy(fine.leaf_n).to(device)
        tl = colden.Tree(fine, ll, max_dirs=w.D)
        del fine
    else:
        raise ValueError(f"a 2^{tin.max_level} field cannot label a network for 2^{leaf_level} grids")
    probe = colden.Surrogate(w.D, 16, colden.CD_SURR_FP32, 0, norm=(0.0, 1.0, 0.0, 1.0), leaf_level=leaf_level)
    T_rows = torch.empty((colden.Surrogate.ROWS, probe.Dout), dtype=torch.float32, device=device)
    probe.row_targets(tl, w, T_rows)
    torch.cuda.synchronize(device)
    probe.close()
    if tl is not tree:
        tl.close()
        del ll
    rng = np.random.default_rng(seed)
    ln_n = np.log(np.maximum(tin.leaf_n[rng.integers(0, tin.n_leaf, ln_sample)].astype(np.float64), 1e-10))
    return LabelledField(tree, leaf, T_rows, ln_n)


def norms(fields, sample_rows: int = 8192, seed: int = 0) -> tuple:
    """Input and output normalisation (in_shift, in_scale, out_shift,
    out_scale) from the training data.  Inputs: centred on the mean ln n of
    the training leaves, scaled so that the out-of-box value ln 1e-10 lands
    at -4 (or by the spread of ln n if that is wider).  Outputs: mean and
    spread of the unscaled targets ln(E + 1e17) over a sample of rows of
    each field's table."""
    import torch

    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    ln_e = []
    for f in fields:
        rows = torch.randint(0, colden.Surrogate.ROWS, (sample_rows,), generator=g).to(f.T_rows.device)
        ln_e.append(f.T_rows[rows].cpu().numpy().astype(np.float64).ravel())
    ln_n = np.concatenate([f.ln_n for f in fields])
    ln_e = np.concatenate(ln_e)
    mu = float(ln_n.mean())
    sc = max(float(ln_n.std()), (mu - np.log(1e-10)) / 4.0)
    return (mu, sc, float(ln_e.mean()), float(max(ln_e.std(), 1e-3)))


def fit(surr: colden.Surrogate, fields, steps: int, batch: int = 4096, lr: float = 2e-3, lr_final: float = 1e-4,
        seed: int = 0, log_every: int = 0):
    """`steps` Adam steps, cycling over the fields, each on `batch` random
    level-7 cells; learning rate decays geometrically from lr to lr_final.
    Returns the logged (step, loss) pairs."""
    import torch

    dev = fields[0].T_rows.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    log = []
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    for k in range(steps):
        f = fields[k % len(fields)]
        rows = torch.randint(0, colden.Surrogate.ROWS, (batch,), device=dev, generator=gen, dtype=torch.int64)
        want = log_every > 0 and (k % log_every == 0 or k == steps - 1)
        loss = surr.train_step_rows(f.tree, f.T_rows, rows, lr * decay ** k, want_loss=want)
        if want:
            if not math.isfinite(loss):
                raise FloatingPointError(f"surrogate loss {loss} at step {k}")
            log.append((k, loss))
    return log
