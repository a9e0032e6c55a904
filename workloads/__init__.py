"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Random numbers and problem definitions only: nothing in this module
computes any part of the solve.

Configurations (per axis: order n, elements K, box length X):
  small_2d    N=2, n=2, K=16, X=(1,1), alpha=0          (31^2 = 961 unknowns)
  large_2d    N=2, n=9, K=1024, X=(1,1), alpha=0        (9215^2 = 84,916,225 unknowns)
  cube_3d     N=3, n=4, K=128, X=(1,1,1), alpha=0       (511^3 = 133,432,831 unknowns)
  varcoef_3d  N=3, n=3, K=64, X=(1,1,1), alpha=0        (191^3 = 6,967,871 unknowns) with
              a(x) = 1 + 0.5 prod_i sin(2 pi k_i x_i), k_i uniform on {1, 2, 3} from the
              seed (variable-coefficient problem -div(a grad u) = f)
  batch_2d    256 independent 2D problems on [0,1]^2, alpha=0, per problem K uniform on
              {32, 64, 128, 256} then n uniform on {2..6}, 4 right-hand sides each
Right-hand sides of the random kind are i.i.d. uniform[-1, 1) values of f^h
drawn in C order with numpy's default generator (PCG64) from the seed.
"""
import numpy as np

CONFIGS = {
    "small_2d": dict(orders=(2, 2), Ks=(16, 16), X=(1.0, 1.0), alpha=0.0),
    "large_2d": dict(orders=(9, 9), Ks=(1024, 1024), X=(1.0, 1.0), alpha=0.0),
    "cube_3d": dict(orders=(4, 4, 4), Ks=(128, 128, 128), X=(1.0, 1.0, 1.0), alpha=0.0),
    "varcoef_3d": dict(orders=(3, 3, 3), Ks=(64, 64, 64), X=(1.0, 1.0, 1.0), alpha=0.0),
}


def shape(orders, Ks):
    return tuple(n * K - 1 for n, K in zip(orders, Ks))


def uniform_rhs(shp, seed=0, dtype=np.float64):
    """f^h with i.i.d. uniform[-1, 1) entries."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, shp).astype(dtype)


def normal_noise(shp, sigma, seed=0):
    """i.i.d. N(0, sigma^2) entries (sigma is the standard deviation)."""
    return np.random.default_rng(seed).normal(0.0, sigma, shp)


def wavenumbers(N, seed=0):
    """k_i uniform on {1, 2, 3} (i = 0..N-1) from the seed."""
    return tuple(int(k) for k in np.random.default_rng(seed).integers(1, 4, N))


def sine_coefficient(ks):
    """(c0, c1, [t_i]) of a(x) = c0 + c1 prod_i t_i(x_i) with
    t_i(x) = sin(2 pi k_i x)."""
    return 1.0, 0.5, [(lambda x, k=k: np.sin(2.0 * np.pi * k * x)) for k in ks]


BATCH = dict(count=256, Ks=(32, 64, 128, 256), orders=(2, 3, 4, 5, 6), nrhs=4,
             X=(1.0, 1.0), alpha=0.0)


def batch_problems(count=256, seed=0, Ks=BATCH["Ks"], orders=BATCH["orders"]):
    """(n, K) per problem: for each problem K, then n, from one generator."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        K = int(rng.choice(Ks))
        n = int(rng.choice(orders))
        out.append((n, K))
    return out


def batch_rhs(problems, nrhs=4, seed=0, dtype=np.float64):
    """Right-hand sides of the batch, one (nrhs, m, m) array per problem in
    problem order, i.i.d. uniform[-1, 1) from a generator seeded seed + 1."""
    rng = np.random.default_rng(seed + 1)
    for n, K in problems:
        m = n * K - 1
        yield rng.uniform(-1.0, 1.0, (nrhs, m, m)).astype(dtype)


def grid_points(n, K, X):
    """Coordinates q X / (n K), q = 1..nK-1, of the unknowns along one axis."""
    return np.arange(1, n * K) * (X / (n * K))

