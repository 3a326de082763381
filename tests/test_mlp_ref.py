"""The CPU reference of the pair-scoring MLP is pinned by finite differences (it has no
paper value: the paper has no MLP), and its BF16 rounding by exact values."""
import numpy as np

from oracle import mlp_ref as R


def test_bf16_rounding_exact_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0],
                 dtype=np.float32)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert list(R.bf16(x)) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0]


def _problem(seed=3, M=8):
    rng = np.random.default_rng(seed)
    flat = np.concatenate([rng.normal(0, np.sqrt(2.0 / 8192), 512 * 8192), rng.normal(0, 0.1, 512),
                           rng.normal(0, np.sqrt(2.0 / 512), 256 * 512), rng.normal(0, 0.1, 256),
                           rng.normal(0, np.sqrt(2.0 / 256), 256), rng.normal(0, 0.1, 1)])
    sig = rng.integers(0, 2 ** 63, size=(6, 64), dtype=np.uint64)
    pairs = np.array([(i << 32) | j for i, j in rng.integers(0, 6, size=(M, 2))], dtype=np.uint64)
    y = rng.integers(0, 2, size=M).astype(np.float64)
    return flat, R.pair_inputs(sig, pairs), y


def test_pair_inputs_layout():
    sig = np.zeros((2, 64), dtype=np.uint64)
    sig[0, 0] = 0b1011
    sig[1, 0] = 0b0110
    sig[0, 63] = 1 << 63
    sig[1, 63] = 1 << 63
    x = R.pair_inputs(sig, np.array([(0 << 32) | 1], dtype=np.uint64))[0]
    assert list(x[:4]) == [1, 0, 1, 1]          # XOR bits 0..3
    assert list(x[4096:4100]) == [0, 1, 0, 0]   # AND bits 0..3
    assert x[4095] == 0 and x[8191] == 1


def test_gradients_match_finite_differences():
    flat, X, y = _problem()
    p = R.unflatten(flat)
    _, g, _ = R.loss_and_grads(p, X, y, pos_weight=3.0, bf16_on=False)
    gflat = R.flatten(g)
    rng = np.random.default_rng(7)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in R.SHAPES])
    idx = []
    for t in range(len(R.SHAPES)):
        idx += list(rng.integers(offsets[t], offsets[t + 1], size=6))
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp = R.loss_and_grads(R.unflatten(fp), X, y, 3.0, False)[0]
        lm = R.loss_and_grads(R.unflatten(fm), X, y, 3.0, False)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, gflat[i])


def test_adam_matches_closed_form_first_step():
    # first bias-corrected step moves each parameter by -lr * sign(g) (up to eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.01, 0.0])
    q, m1, m2 = R.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(q, p - 0.1 * np.sign(g), atol=1e-6)
