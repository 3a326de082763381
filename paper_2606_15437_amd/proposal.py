"""Learned pair proposal: rank candidate formula pairs by a trained MLP, then verify every
proposal exactly with the census and split kernels.

A *late split* (the retrieval target) is a pair (phi, psi) whose biconditional
phi <-> psi has no countermodel on any frame with at most 4 worlds, while a
separating model exists on the 6-8-world stress panel (Definition 2 and
Proposition 5: the pair is k-indistinguishable for some k >= 4).  The analogue in
the paper is representation-guided retrieval followed by exhaustive rescans
(Section 9); here the representation is a learned scorer over exact
small-model signatures.

Steps (every evaluation runs in the library's kernels):
  1. signatures: truth bits of each formula at 4,096 pointed models (<= 3 worlds);
  2. universe: each formula's k nearest formulas by signature Hamming distance,
     unordered pairs in canonical (i, j) order;
  3. verification of a pair list: census of phi <-> psi over every frame with
     n = 1..4 worlds and every valuation (early exit at the first
     countermodel, survivors carried to the next n), then the first
     separating model on the stress panel (the first frames of the seeded
     6-, 7- and 8-world families);
  4. labels for a separately seeded training corpus from step 3, MLP training
     with BCE-with-logits (positive weight) and Adam;
  5. ranking of the test universe by the MLP (learned), by canonical order
     (plain enumeration) and by signature Hamming distance; the top `budget`
     pairs of each are verified, and hits per 10^6 evaluated pairs reported.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs as I
from . import kripke as K

NVARS = 2


def _t():
    import torch
    return torch


def signatures(formulas, samples=None, device="cuda"):
    torch = _t()
    samples = I.signature_samples() if samples is None else samples
    code, offs = I.pack(formulas)
    d = torch.zeros((len(formulas), len(samples) // 64), dtype=torch.int64, device=device)
    K.kripke_signatures(code, offs, NVARS, samples, d)
    return d


def universe(d_sig, k):
    torch = _t()
    nf = d_sig.shape[0]
    d_pairs = torch.zeros(nf * k, dtype=torch.int64, device=d_sig.device)
    d_n = torch.zeros(1, dtype=torch.int64, device=d_sig.device)
    K.kripke_knn_pairs(d_sig, k, d_pairs, d_n)
    n = int(d_n.item())
    return d_pairs[:n].clone()


def universe_of_size(d_sig, target):
    """The universe for the neighbour count k whose size is closest to target (the size
    grows with k; bisection over k)."""
    nf = d_sig.shape[0]
    lo, hi = 1, nf - 1
    best = None
    while lo <= hi:
        k = (lo + hi) // 2
        u = universe(d_sig, k)
        if best is None or abs(u.shape[0] - target) < abs(best[1].shape[0] - target):
            best = (k, u)
        if u.shape[0] < target:
            lo = k + 1
        elif u.shape[0] > target:
            hi = k - 1
        else:
            break
        del u
    return best


def stress_panel(frames_per_n=4096):
    """The stress panel: frames 0 .. frames_per_n-1 of the seeded families at n = 6, 7, 8."""
    return {n: I.frame_family(n, frames_per_n) for n in (6, 7, 8)}


def _pairs_host(d_pairs):
    p = K.as_u64(d_pairs) if hasattr(d_pairs, "is_cuda") else np.asarray(d_pairs, dtype=np.uint64)
    return (p >> np.uint64(32)).astype(np.int64), (p & np.uint64(0xFFFFFFFF)).astype(np.int64)


class Verifier:
    """Exact verdicts on pairs: agreement through 4 worlds, then a split on the panel."""

    def __init__(self, formulas, panel=None, chunk=1 << 17, log=None):
        torch = _t()
        self.formulas = formulas
        self.panel = stress_panel() if panel is None else panel
        self.d_panel = {n: torch.as_tensor(np.ascontiguousarray(fr).view(np.int32), device="cuda")
                        for n, fr in self.panel.items()}
        self.chunk = chunk
        self.evals = 0.0
        self.log = log
        # wall time and evaluations per stage ("agree n=1", ..., "split n=8"), and
        # for the split stages the executed INT32 lane-operations (Proposition 2's
        # bit-ops of the compiled biconditionals x models scanned / 32)
        self.stage_s = {}
        self.stage_evals = {}
        self.stage_ops = {}
        code, offs = I.pack(formulas)
        self.code = np.concatenate([code, np.array([I.IFF], dtype=np.uint8)])
        self.offs = offs[:-1].astype(np.int64)
        self.lens = np.diff(offs).astype(np.int64)

    def _programs(self, ia, ib, chi):
        """CSR batch of phi_k <-> psi_k (chi=True) or of phi_0, psi_0, phi_1, ... built by
        gathering from the packed corpus."""
        la = self.lens[ia]
        lb = self.lens[ib]
        per = la + lb + (1 if chi else 0)
        offs = np.zeros(len(ia) + 1, dtype=np.int64)
        np.cumsum(per, out=offs[1:])
        total = int(offs[-1])
        pid = np.repeat(np.arange(len(ia)), per)
        local = np.arange(total, dtype=np.int64) - offs[pid]
        src = np.where(local < la[pid], self.offs[ia][pid] + local,
                       np.where(local < (la + lb)[pid], self.offs[ib][pid] + local - la[pid],
                                len(self.code) - 1))
        code = self.code[src]
        if chi:
            return code, offs.astype(np.uint32)
        split = np.empty(2 * len(ia) + 1, dtype=np.int64)
        split[0::2] = offs
        split[1::2] = offs[:-1] + la
        return code, split.astype(np.uint32)

    def _stage(self, name, t0, evals):
        self.stage_s[name] = self.stage_s.get(name, 0.0) + time.time() - t0
        self.stage_evals[name] = self.stage_evals.get(name, 0.0) + evals
        self.evals += evals

    def _bitops(self, ia, ib, n):
        """Executed bit-ops per evaluation of each pair's compiled biconditional."""
        code, offs = self._programs(ia, ib, True)
        st = K.kripke_program_stats(code, offs, NVARS)
        return n * st[:, 1].astype(np.float64) + n * n * st[:, 0].astype(np.float64)

    def stage_rates(self):
        """INT32 lane-operations per second of each split stage (frames up to the
        separating one, else all; the stage's wall time includes host compilation)."""
        return {k: self.stage_ops[k] / self.stage_s[k] / 1e12 for k in self.stage_s
                if self.stage_s[k] > 0 and self.stage_ops.get(k)}

    def agree_through(self, ia, ib, nmax=4, layers=None):
        """Mask of pairs whose biconditional has no countermodel on any frame with
        n <= nmax worlds (census with early exit, survivors only per layer); `layers`
        restricts the check to the given layers.  The evaluation count is an upper bound
        (every scanned layer counted in full)."""
        torch = _t()
        alive = np.ones(len(ia), dtype=bool)
        for n in (range(1, nmax + 1) if layers is None else layers):
            t0 = time.time()
            idx = np.nonzero(alive)[0]
            for s in range(0, len(idx), self.chunk):
                sub = idx[s:s + self.chunk]
                code, offs = self._programs(ia[sub], ib[sub], True)
                out = torch.empty((len(sub), 2), dtype=torch.int64, device="cuda")
                K.kripke_census_range(code, offs, n, K.KRIPKE_K, NVARS, 0, 1 << (n * n),
                                      K.KRIPKE_DECIDE, out)
                keys = K.as_u64(out)[:, 0]
                alive[sub] = keys == K.NO_KEY
            self._stage(f"agree n={n}", t0, float(len(idx)) * (1 << (n * n)) * (1 << (NVARS * n)))
            if self.log:
                self.log(f"  agree n={n}: {len(idx)} in, {int(alive.sum())} agree "
                         f"({self.stage_s[f'agree n={n}']:.2f} s)")
        return alive

    def split_keys(self, ia, ib):
        """First separating key on the panel (n = 6, 7, 8 in turn), or NO_KEY."""
        torch = _t()
        found = np.full(len(ia), K.NO_KEY, dtype=np.uint64)
        where = np.zeros(len(ia), dtype=np.int64)
        for n in (6, 7, 8):
            t0 = time.time()
            idx = np.nonzero(found == K.NO_KEY)[0]
            for s in range(0, len(idx), self.chunk):
                sub = idx[s:s + self.chunk]
                code, offs = self._programs(ia[sub], ib[sub], False)
                out = torch.empty(len(sub), dtype=torch.int64, device="cuda")
                K.kripke_split_batch(code, offs, self.d_panel[n], n, NVARS, out)
                k = K.as_u64(out)
                found[sub] = k
                where[sub[k != K.NO_KEY]] = n
            self._stage(f"split n={n}", t0,
                        float(len(idx)) * len(self.panel[n]) * (1 << (NVARS * n)))
            if len(idx):  # executed work, counted outside the stage's time
                k = found[idx]
                scanned = np.where(k != K.NO_KEY,
                                   (k >> np.uint64(NVARS * n + 4)).astype(np.float64) + 1,
                                   float(len(self.panel[n])))
                self.stage_ops[f"split n={n}"] = self.stage_ops.get(f"split n={n}", 0.0) + float(
                    (self._bitops(ia[idx], ib[idx], n) * scanned).sum()) * (1 << (NVARS * n)) / 32.0
            if self.log:
                self.log(f"  split n={n}: {len(idx)} in, {int((where == n).sum())} split "
                         f"({self.stage_s[f'split n={n}']:.2f} s)")
        return found, where

    def verify(self, d_pairs_or_host):
        """Per pair: 1 if it is a late split (agrees through 4 worlds, splits on the panel)."""
        ia, ib = _pairs_host(d_pairs_or_host)
        hit = np.zeros(len(ia), dtype=bool)
        agree = self.agree_through(ia, ib)
        idx = np.nonzero(agree)[0]
        keys = np.full(len(ia), K.NO_KEY, dtype=np.uint64)
        where = np.zeros(len(ia), dtype=np.int64)
        if len(idx):
            k, w = self.split_keys(ia[idx], ib[idx])
            keys[idx], where[idx] = k, w
            hit[idx] = k != K.NO_KEY
        return hit, {"agree4": agree, "keys": keys, "n": where}


# Pairs per forward chunk when scoring a universe: large enough that the first
# layer's GEMM runs with its widest per-wave tiles (they need a grid of at least 1,024
# blocks of 128 x 256 outputs, i.e. 65,536 or more pairs per chunk).
SCORE_CHUNK = 1 << 18


def train_mlp(d_sig, d_pairs, labels, steps=400, batch=512, lr=1e-3, seed=17, log=None):
    """Train the scorer on labelled pairs (balanced sampling is left to pos_weight)."""
    torch = _t()
    n = d_pairs.shape[0]
    pos = float(labels.sum())
    pos_weight = float((n - pos) / max(pos, 1.0))
    d_y_all = torch.as_tensor(labels.astype(np.float32), device="cuda")
    h = K.kripke_mlp_create(seed, max(batch, SCORE_CHUNK))
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    losses = []
    for step in range(steps):
        sel = torch.as_tensor(rng.integers(0, n, size=batch), device="cuda")
        K.kripke_mlp_gradients(h, d_sig, d_pairs[sel].contiguous(), d_y_all[sel].contiguous(),
                               pos_weight, d_loss)
        K.kripke_mlp_adam_step(h, lr=lr)
        if step % 50 == 0 or step == steps - 1:
            losses.append(float(d_loss.item()))
            if log:
                log(f"train step {step}: loss {losses[-1]:.4f}")
    return h, losses, pos_weight


def score(h, d_sig, d_pairs):
    torch = _t()
    d_z = torch.empty(d_pairs.shape[0], dtype=torch.float32, device="cuda")
    K.kripke_mlp_forward(h, d_sig, d_pairs, d_z)
    return d_z


def top(d_scores, budget):
    torch = _t()
    b = min(budget, d_scores.numel())
    d_idx = torch.empty(b, dtype=torch.int64, device="cuda")
    K.kripke_select_top(d_scores, b, d_idx)
    return d_idx


def hamming_scores(d_sig, d_pairs):
    torch = _t()
    d = torch.empty(d_pairs.shape[0], dtype=torch.int32, device="cuda")
    K.kripke_pair_hamming(d_sig, d_pairs, d_pairs.shape[0], d)
    return -d.float()


def run(n_test=10000, n_train=10000, universe_pairs=5_500_000, train_pairs=5_500_000,
        budget=1_000_000, steps=2000, panel_frames=4096, log=print, details=False):
    """The full protocol; returns a dict of hit counts and timings.  With details, also
    the verified pairs (host arrays) under "details": canonical pair codes of the verified
    union and their (sorted) indices in the test universe, hit flags, agreement flags,
    separating keys, the n they were found at, and each ranking as universe indices."""
    torch = _t()
    t0 = time.time()
    rec = {}
    train = I.retrieval_corpus(I.SEED_C5_TRAIN, n_train, n_words=n_train // 5)
    test = I.retrieval_corpus(I.SEED_C5_TEST, n_test, n_words=n_test // 5)
    panel = stress_panel(panel_frames)
    # training labels
    s_tr = signatures(train)
    k_train, u_tr = universe_of_size(s_tr, train_pairs)
    log(f"training universe {u_tr.shape[0]} pairs ({time.time() - t0:.1f} s)")
    ver_tr = Verifier(train, panel, log=log)
    lab, _ = ver_tr.verify(u_tr)
    rec["train"] = {"formulas": n_train, "k": k_train, "pairs": int(u_tr.shape[0]),
                    "positives": int(lab.sum()),
                    "label_evals": ver_tr.evals, "label_s": time.time() - t0,
                    "label_stages_s": dict(ver_tr.stage_s)}
    log(f"training labels: {int(lab.sum())} late splits ({time.time() - t0:.1f} s)")
    t1 = time.time()
    h, losses, pw = train_mlp(s_tr, u_tr, lab, steps=steps, log=log)
    rec["train"].update({"steps": steps, "loss": losses, "pos_weight": pw,
                         "train_s": time.time() - t1})
    # test universe
    s_te = signatures(test)
    k_test, u_te = universe_of_size(s_te, universe_pairs)
    npairs = int(u_te.shape[0])
    rec["test"] = {"formulas": n_test, "k": k_test, "pairs": npairs, "budget": budget}
    log(f"test universe {npairs} pairs (k={k_test})")
    ver = Verifier(test, panel, log=log)
    rankings = {}
    t2 = time.time()
    z = score(h, s_te, u_te)
    torch.cuda.synchronize()
    rec["test"]["score_s"] = time.time() - t2
    rankings["learned"] = top(z, budget)
    rankings["plain"] = torch.arange(min(budget, npairs), device="cuda")
    rankings["hamming"] = top(hamming_scores(s_te, u_te), budget)
    # verify the union once, then count per ranking
    union = torch.unique(torch.cat([r for r in rankings.values()]))
    t3 = time.time()
    hit_u, info = ver.verify(u_te[union])
    rec["test"]["verify_s"] = time.time() - t3
    rec["test"]["verify_evals"] = ver.evals
    union_h = union.cpu().numpy()  # sorted
    for name, r in rankings.items():
        ids = r.cpu().numpy()
        hit = hit_u[np.searchsorted(union_h, ids)]
        hits = int(hit.sum())
        # every ranking is stable, so a smaller budget's selection is a prefix
        prefix = {str(b): int(hit[:b].sum()) for b in (10_000, 100_000) if b < len(ids)}
        # the smallest budget at which this ranking holds a given share of every late
        # split verified in the union of the rankings (None if it never does)
        total = int(hit_u.sum())
        cum = np.cumsum(hit)
        reach = {}
        for share in (0.5, 0.9):
            need = int(np.ceil(share * total))
            at = int(np.searchsorted(cum, need)) if need else 0
            reach[str(share)] = at + 1 if total and at < len(cum) else None
        rec[name] = {"evaluated": int(len(ids)), "hits": hits,
                     "hits_per_1e6": hits * 1e6 / max(len(ids), 1), "hits_at_budget": prefix,
                     "budget_for_share_of_all_hits": reach}
        log(f"{name}: {hits} verified late splits in {len(ids)} pairs; at smaller budgets "
            f"{prefix}")
    rec["test"]["verify_stages_s"] = dict(ver.stage_s)
    rec["test"]["verify_stage_evals"] = dict(ver.stage_evals)
    rec["test"]["verify_stage_T_int32_ops_per_s"] = ver.stage_rates()
    # the paper's stricter hit (Section 9): the biconditional also has no countermodel on
    # any frame with five worlds (every labelled frame, every valuation)
    t4 = time.time()
    hit_idx = np.nonzero(hit_u)[0]
    ia_u, ib_u = _pairs_host(u_te[union])
    agree5 = np.zeros(len(hit_u), dtype=bool)
    if len(hit_idx):
        agree5[hit_idx] = ver.agree_through(ia_u[hit_idx], ib_u[hit_idx], layers=(5,))
    rec["test"]["five_world_s"] = time.time() - t4
    for name, r in rankings.items():
        ids = np.searchsorted(union_h, r.cpu().numpy())
        rec[name]["hits_five_world"] = int(agree5[ids].sum())
        log(f"{name}: {rec[name]['hits_five_world']} of its hits also agree on every "
            f"five-world model")
    rec["hits_detail"] = {"union": int(union.numel()), "agree4": int(info["agree4"].sum()),
                          "late_splits": int(hit_u.sum()),
                          "late_splits_five_world": int(agree5.sum())}
    if details:
        rec["details"] = {"pairs": K.as_u64(u_te[union]).copy(), "union_idx": union_h,
                          "hit": hit_u,
                          "agree5": agree5,
                          "agree4": info["agree4"], "keys": info["keys"], "n": info["n"],
                          "panel": panel, "rankings": {k: v.cpu().numpy()
                                                       for k, v in rankings.items()}}
    rec["total_s"] = time.time() - t0
    K.kripke_mlp_destroy(h)
    return rec
