"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no homomorphic arithmetic: it only draws data (numpy PCG64)
and names the workload sizes.  Both the GPU path and the CPU oracle take their
inputs from here.

Stand-ins (the paper's data sets are not available):
  * small   -- 2048 x 16 features uniform in [-1,1], labels from a seeded
               random linear model with 5% flipped labels;
  * image   -- two-class, 14x14 "digit-like" images (the paper's MNIST 3-vs-8
               at 14x14, Sec. 5.1), 6000 samples for one server's shard:
               seeded Gaussian blobs per class, values in [0,1], 80% zeros;
  * large   -- 2^20 x 512 dense Gaussian, labels from a random linear model
               with 10% flips.
"""
import numpy as np

WORKLOADS = {
    # ring degree, ciphertext primes, special primes, primes per digit, log2 scale
    "small": dict(logN=13, nq=5, nk=1, alpha=1, log_delta=30, n=2048, d=16, steps=1,
                  refresh=0, seed_data=1001, seed_keys=2001, seed_enc=3001, seed_w=4001),
    "image": dict(logN=16, nq=20, nk=4, alpha=4, log_delta=40, n=6000, d=196, steps=10,
                  refresh=4, seed_data=1002, seed_keys=2002, seed_enc=3002, seed_w=4002),
    "large": dict(logN=16, nq=24, nk=6, alpha=6, log_delta=40, n=1 << 20, d=512, steps=5,
                  refresh=0, seed_data=1005, seed_keys=2005, seed_enc=3005, seed_w=4005),
}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _flip(g, y, frac):
    n = y.shape[0]
    k = int(round(frac * n))
    idx = g.permutation(n)[:k]
    y = y.copy()
    y[idx] = -y[idx]
    return y


def small_data(seed=1001, n=2048, d=16):
    g = rng(seed)
    X = g.uniform(-1.0, 1.0, size=(n, d))
    w_star = g.standard_normal(d)
    y = np.where(X @ w_star >= 0, 1.0, -1.0)
    return X, _flip(g, y, 0.05)


def image_data(seed=1002, n=6000, side=14):
    """Two classes of n/2 images; each class has 4 blob centres in [3,10]^2;
    an image sums 2 of its class's blobs, amp ~ U[0.6,1], width ~ U[1,2] px,
    offset ~ N(0,1) px, clipped to [0,1]; pixels below the image's 80th
    percentile are set to zero."""
    g = rng(seed)
    centres = g.uniform(3.0, 10.0, size=(2, 4, 2))
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    X = np.zeros((n, side * side))
    y = np.zeros(n)
    for i in range(n):
        cls = i % 2
        img = np.zeros((side, side))
        for k in g.choice(4, size=2, replace=False):
            amp = g.uniform(0.6, 1.0)
            sig = g.uniform(1.0, 2.0)
            mu = centres[cls, k] + g.standard_normal(2)
            img += amp * np.exp(-((yy - mu[0]) ** 2 + (xx - mu[1]) ** 2) / (2 * sig * sig))
        img = np.clip(img, 0.0, 1.0)
        thr = np.percentile(img, 80)
        img[img < thr] = 0.0
        X[i] = img.ravel()
        y[i] = 1.0 if cls == 0 else -1.0
    perm = g.permutation(n)
    return X[perm], y[perm]


def large_block(seed, block, rows, d=512):
    """Rows [block*rows, (block+1)*rows) of the large workload, drawn per block
    so that no more than one block is ever held in memory."""
    g0 = rng(seed)
    w_star = g0.standard_normal(d) / np.sqrt(d)
    g = rng(seed * 1000003 + block)
    X = g.standard_normal((rows, d))
    y = np.where(X @ w_star >= 0, 1.0, -1.0)
    flip = g.uniform(size=rows) < 0.10
    y[flip] = -y[flip]
    return X, y


def initial_weights(name, d, seed):
    if name == "small":
        return rng(seed).uniform(-0.25, 0.25, size=d)
    return np.zeros(d)


def uniform_residues(seed, primes, N):
    """Independent uniform residues, one row per prime: [len(primes)][N] uint64."""
    g = rng(seed)
    return np.stack([g.integers(0, q, size=N, dtype=np.uint64) for q in primes])


def small_poly(seed, N, bound):
    """Integer polynomial with coefficients uniform in [-bound, bound]."""
    return rng(seed).integers(-bound, bound + 1, size=N, dtype=np.int64)
