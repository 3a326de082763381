"""GPU tests of the learned-proposal path: signatures against the oracle, candidate
pairs and rankings against brute force written here, and the MFMA MLP against the CPU
reference (forward, gradients, Adam) plus a training sanity check."""
import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _sig_gpu(kr, formulas, samples):
    import torch
    code, offs = I.pack(formulas)
    d = torch.zeros((len(formulas), len(samples) // 64), dtype=torch.int64, device="cuda")
    kr.kripke_signatures(code, offs, 2, samples, d)
    torch.cuda.synchronize()
    return kr.as_u64(d)


def test_signatures_match_oracle(kr, orc):
    samples = I.signature_samples()
    fs = I.retrieval_corpus(I.SEED_C5_TEST, 300, n_words=120)
    got = _sig_gpu(kr, fs, samples)
    exp = orc.signatures(fs, samples, 2)
    assert (got == exp).all()


def test_signatures_reject_mixed_groups(kr):
    import torch
    samples = I.signature_samples().copy()
    samples[5] = (2 << 60) | (1 << 24) | (0 << 4) | 0  # a 2-world model inside a 3-world group
    code, offs = I.pack([[I.TOP]])
    d = torch.zeros((1, 64), dtype=torch.int64, device="cuda")
    with pytest.raises(kr.KripkeError):
        kr.kripke_signatures(code, offs, 2, samples, d)


def _brute_knn_pairs(sig, k):
    nf = len(sig)
    d = np.zeros((nf, nf), dtype=np.int64)
    for i in range(nf):
        x = sig[i] ^ sig
        d[i] = np.unpackbits(x.view(np.uint8), axis=1).sum(1)
    pairs = set()
    for i in range(nf):
        order = sorted((int(d[i, j]), j) for j in range(nf) if j != i)[:k]
        for _, j in order:
            pairs.add((min(i, j), max(i, j)))
    return sorted(pairs), d


def test_knn_pairs_and_hamming(kr):
    import torch
    rng = np.random.default_rng(11)
    nf, k = 300, 17
    # clustered signatures so that ties and asymmetric neighbourhoods occur
    base = rng.integers(0, 2 ** 63, size=(20, 64), dtype=np.uint64)
    sig = base[rng.integers(0, 20, size=nf)].copy()
    flips = rng.integers(0, 4096, size=(nf, 3))
    for i in range(nf):
        for b in flips[i]:
            sig[i, b // 64] ^= np.uint64(1) << np.uint64(b % 64)
    d_sig = torch.as_tensor(sig.view(np.int64), device="cuda")
    d_pairs = torch.zeros(nf * k, dtype=torch.int64, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    kr.kripke_knn_pairs(d_sig, k, d_pairs, d_n)
    torch.cuda.synchronize()
    npairs = int(d_n.item())
    got = kr.as_u64(d_pairs)[:npairs]
    exp, dist = _brute_knn_pairs(sig, k)
    assert [(int(p >> 32), int(p & 0xFFFFFFFF)) for p in got] == exp
    d_dist = torch.zeros(npairs, dtype=torch.int32, device="cuda")
    kr.kripke_pair_hamming(d_sig, d_pairs, npairs, d_dist)
    torch.cuda.synchronize()
    assert list(d_dist.cpu().numpy()) == [int(dist[i, j]) for i, j in exp]


def test_select_top_stable(kr):
    import torch
    rng = np.random.default_rng(5)
    s = rng.integers(-20, 20, size=5000).astype(np.float32) / 4
    s[::7] = 0.0
    s[3::11] = -0.0
    d_s = torch.as_tensor(s, device="cuda")
    d_i = torch.zeros(1000, dtype=torch.int64, device="cuda")
    kr.kripke_select_top(d_s, 1000, d_i)
    torch.cuda.synchronize()
    exp = sorted(range(len(s)), key=lambda i: (-float(s[i]) if s[i] != 0 else 0.0, i))[:1000]
    assert list(d_i.cpu().numpy()) == exp


# ----------------------------------------------------------------- MLP
def _mlp_problem(kr, M=128, seed=9):
    import torch
    rng = np.random.default_rng(seed)
    sig = rng.integers(0, 2 ** 63, size=(40, 64), dtype=np.uint64)
    ij = rng.integers(0, 40, size=(M, 2))
    pairs = np.array([(int(i) << 32) | int(j) for i, j in ij], dtype=np.uint64)
    y = (rng.random(M) < 0.3).astype(np.float32)
    d_sig = torch.as_tensor(sig.view(np.int64), device="cuda")
    d_pairs = torch.as_tensor(pairs.view(np.int64), device="cuda")
    d_y = torch.as_tensor(y, device="cuda")
    return sig, pairs, y, d_sig, d_pairs, d_y


def _close(got, exp, rel):
    scale = max(float(np.max(np.abs(exp))), 1e-12)
    return float(np.max(np.abs(got - exp))) <= rel * scale


def test_mlp_forward_matches_reference(kr):
    import torch
    from oracle import mlp_ref as R
    sig, pairs, y, d_sig, d_pairs, d_y = _mlp_problem(kr, M=200)
    h = kr.kripke_mlp_create(1234, 128)
    try:
        # non-zero biases so every term of the epilogues is exercised
        p = kr.kripke_mlp_get_params(h)
        rng = np.random.default_rng(1)
        named = kr.split_params(p)
        for b in ("b1", "b2", "b3"):
            named[b][:] = rng.normal(0, 0.05, named[b].shape)
        kr.kripke_mlp_set_params(h, p)
        d_z = torch.zeros(len(pairs), dtype=torch.float32, device="cuda")
        kr.kripke_mlp_forward(h, d_sig, d_pairs, d_z)  # 200 pairs: two chunks of <= 128
        torch.cuda.synchronize()
        ref = R.forward(R.unflatten(p), R.pair_inputs(sig, pairs))["z"]
        assert _close(d_z.cpu().numpy(), ref, 1e-2)
    finally:
        kr.kripke_mlp_destroy(h)


def test_mlp_wide_tiles_match_narrow_and_reference(kr):
    """A forward of 65,728 pairs in one chunk runs the first layer on the LDS-staged
    kernel (256 pairs x 128 outputs per block, 2 x 4 MFMA tiles per wave; 257 row
    blocks, so the last one is ragged and the grid has a padding block) and the second
    with 2 x 2 tiles per wave, as the scoring path's chunks do; it equals, bit for bit,
    the same pairs forwarded in chunks of 512 (one tile per wave), and sampled rows match
    the CPU reference."""
    import torch
    from oracle import mlp_ref as R
    rng = np.random.default_rng(21)
    sig = rng.integers(0, 2 ** 63, size=(300, 64), dtype=np.uint64)
    M = 65536 + 192
    ij = rng.integers(0, 300, size=(M, 2))
    pairs = (ij[:, 0].astype(np.uint64) << np.uint64(32)) | ij[:, 1].astype(np.uint64)
    d_sig = torch.as_tensor(sig.view(np.int64), device="cuda")
    d_pairs = torch.as_tensor(pairs.view(np.int64), device="cuda")
    wide = kr.kripke_mlp_create(31, M)
    narrow = kr.kripke_mlp_create(31, 512)
    try:
        p = kr.kripke_mlp_get_params(wide)
        named = kr.split_params(p)
        for b in ("b1", "b2", "b3"):
            named[b][:] = rng.normal(0, 0.05, named[b].shape)
        kr.kripke_mlp_set_params(wide, p)
        kr.kripke_mlp_set_params(narrow, p)
        z_w = torch.zeros(M, dtype=torch.float32, device="cuda")
        z_n = torch.zeros(M, dtype=torch.float32, device="cuda")
        kr.kripke_mlp_forward(wide, d_sig, d_pairs, z_w)
        kr.kripke_mlp_forward(narrow, d_sig, d_pairs, z_n)
        torch.cuda.synchronize()
        zw, zn = z_w.cpu().numpy(), z_n.cpu().numpy()
        assert (zw.view(np.uint32) == zn.view(np.uint32)).all()
        rows = np.concatenate([rng.choice(M, 96, replace=False), np.arange(M - 8, M)])
        ref = R.forward(R.unflatten(p), R.pair_inputs(sig, pairs[rows]))["z"]
        assert _close(zw[rows], ref, 1e-2)
    finally:
        kr.kripke_mlp_destroy(wide)
        kr.kripke_mlp_destroy(narrow)


def test_mlp_gradients_and_adam_match_reference(kr):
    import torch
    from oracle import mlp_ref as R
    sig, pairs, y, d_sig, d_pairs, d_y = _mlp_problem(kr, M=128)
    h = kr.kripke_mlp_create(77, 256)
    try:
        p = kr.kripke_mlp_get_params(h)
        d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        kr.kripke_mlp_gradients(h, d_sig, d_pairs, d_y, 2.5, d_loss)
        torch.cuda.synchronize()
        g = kr.split_params(kr.kripke_mlp_get_grads(h))
        X = R.pair_inputs(sig, pairs)
        loss, gr, _ = R.loss_and_grads(R.unflatten(p), X, y.astype(np.float64), 2.5, bf16_on=True)
        assert abs(float(d_loss.item()) - loss) <= 1e-4 * max(1.0, abs(loss))
        for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
            assert _close(g[name], gr[name], 2e-2), name
        # one Adam step from the GPU's own gradients equals the reference step
        gflat = kr.kripke_mlp_get_grads(h).astype(np.float64)
        kr.kripke_mlp_adam_step(h, lr=1e-3)
        torch.cuda.synchronize()
        q = kr.kripke_mlp_get_params(h)
        qr, _, _ = R.adam(p.astype(np.float64), gflat, np.zeros_like(gflat), np.zeros_like(gflat), 1,
                          lr=1e-3)
        assert np.max(np.abs(q - qr)) <= 1e-6
    finally:
        kr.kripke_mlp_destroy(h)


def test_mlp_training_reduces_loss(kr):
    """A learnable task: label = 1 iff the XOR half of the input is empty in the first word
    (pairs equal there).  Twenty Adam steps must cut the loss substantially."""
    import torch
    rng = np.random.default_rng(3)
    sig = rng.integers(0, 2 ** 63, size=(64, 64), dtype=np.uint64)
    sig[32:, 0] = sig[:32, 0]
    ij = rng.integers(0, 64, size=(512, 2))
    ij[::2, 1] = (ij[::2, 0] + 32) % 64
    pairs = np.array([(int(i) << 32) | int(j) for i, j in ij], dtype=np.uint64)
    y = np.array([float(sig[i, 0] == sig[j, 0]) for i, j in ij], dtype=np.float32)
    d_sig = torch.as_tensor(sig.view(np.int64), device="cuda")
    d_pairs = torch.as_tensor(pairs.view(np.int64), device="cuda")
    d_y = torch.as_tensor(y, device="cuda")
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    h = kr.kripke_mlp_create(5, 512)
    try:
        losses = []
        for _ in range(20):
            kr.kripke_mlp_gradients(h, d_sig, d_pairs, d_y, 1.0, d_loss)
            kr.kripke_mlp_adam_step(h, lr=1e-3)
            torch.cuda.synchronize()
            losses.append(float(d_loss.item()))
        assert losses[-1] < 0.5 * losses[0], losses
    finally:
        kr.kripke_mlp_destroy(h)


# ------------------------------------------------------------ pipeline
def test_learned_ranking_beats_plain_and_hits_are_certified(kr, orc):
    """The protocol at reduced scale: the learned ranking finds more verified late splits
    than plain canonical enumeration and than the signature Hamming ranking at equal
    budget, and the oracle confirms a sample of
    the verdicts: a hit agrees through 4 worlds and its key is the panel's first
    separating model; a rejected pair has a countermodel within 4 worlds; a pair the
    panel does not separate has no separating model on the 6-world panel nor on the
    first frames of the 7- and 8-world panels (the full panels cost the oracle minutes)."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2606_15437_amd import proposal as P
    rec = P.run(n_test=2000, n_train=2000, universe_pairs=300_000, train_pairs=200_000,
                budget=20_000, steps=300, panel_frames=256, log=lambda m: None, details=True)
    assert rec["learned"]["hits"] > 2 * rec["plain"]["hits"], rec
    d = rec["details"]
    # hits of each ranking within its first b proposals (rankings are stable, so a
    # smaller budget's selection is a prefix)
    at = {}
    for name, ids in d["rankings"].items():
        hit = d["hit"][np.searchsorted(d["union_idx"], ids)]
        at[name] = {b: int(hit[:b].sum()) for b in (500, 1000, 2000, 5000, 10000, 20000)}
    print("hits at budget:", at, flush=True)
    # the trained scorer also ranks ahead of the signature-distance baseline: it holds at
    # least as many hits at every budget up to 10^4 and a clear margin at 5,000 (measured:
    # 565 against 383; every step of the protocol is seeded and deterministic)
    for b in (500, 1000, 2000, 5000, 10000):
        assert at["learned"][b] >= at["hamming"][b], (b, at)
    assert at["learned"][5000] > 1.2 * at["hamming"][5000], at
    test = I.retrieval_corpus(I.SEED_C5_TEST, 2000, n_words=400)
    ia = (d["pairs"] >> np.uint64(32)).astype(np.int64)
    ib = (d["pairs"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    hits = np.nonzero(d["hit"])[0][:16]
    quiet = np.nonzero(d["agree4"] & ~d["hit"])[0][:3]
    late = np.nonzero(~d["agree4"])[0][:16]
    assert len(hits) >= 10 and len(quiet) == 3

    def check_hit(x):
        a, b = test[ia[x]], test[ib[x]]
        chi = I.iff(a, b)
        for n in (1, 2, 3, 4):
            if orc.census(chi, n, 0, 2, stop_at_first=True)[0] != orc.NONE:
                return False
        n = int(d["n"][x])
        frames = d["panel"][n]
        pos, val, world = orc.decode_key(int(d["keys"][x]), n, 2)
        # the key is the first separating model on the panel at the first n that has one
        return orc.split(a, b, frames, 2) == int(d["keys"][x]) and \
            orc.sat_at(a, frames[pos], 2, val, world) != orc.sat_at(b, frames[pos], 2, val, world)

    def check_quiet(x):
        a, b = test[ia[x]], test[ib[x]]
        return all(orc.split(a, b, d["panel"][n][:m], 2) == orc.NONE
                   for n, m in ((6, 256), (7, 48), (8, 12)))

    def check_early(x):
        chi = I.iff(test[ia[x]], test[ib[x]])
        return any(orc.census(chi, n, 0, 2, stop_at_first=True)[0] != orc.NONE
                   for n in (1, 2, 3, 4))

    with ThreadPoolExecutor(max_workers=16) as ex:
        assert all(ex.map(check_hit, hits))
        assert all(ex.map(check_quiet, quiet))
        assert all(ex.map(check_early, late))
