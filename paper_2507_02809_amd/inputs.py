"""Seeded synthetic inputs for the inverse-source problem.

This module only draws and samples inputs; it holds none of the solver's
arithmetic (no time weights, no stencil, no operator).  Both the GPU path's
tests/bench and the CPU oracle read their inputs from here so that they see
bit-identical arrays.

An input set carries the scalar parameters of the problem and the sampled
fields on the grid x_j = j * length/(N+1), j = 1..N per direction (interior
points of Omega = (0, length)^d), t_s = s*T/M, s = 1..M:

  gamma1, gamma2 : (M, N^d)  coefficient samples at (x_j, t_s)
  q              : (M,)      q(t_s)
  rho            : (N^d,)    initial state
  f_true         : (N^d,)    the source used to make the final-time data
  noise          : (N^d,)    noise pattern; the noisy data is
                             mu_eps = mu + noise_level * ||mu||_2 * noise
                             where mu is the final-time state of the forward
                             problem driven by f_true.

Random draws use numpy's default_rng([250702809, config_id, instance]) in a
fixed order: coefficient amplitudes, source modes, noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 250702809


@dataclasses.dataclass
class Inputs:
    name: str
    d: int
    N: int
    M: int
    T: float
    beta: float
    omega: float
    alpha: float
    length: float
    gamma1: np.ndarray
    gamma2: np.ndarray
    q: np.ndarray
    rho: np.ndarray
    f_true: np.ndarray
    noise: np.ndarray
    noise_level: float

    @property
    def Nd(self) -> int:
        return self.N ** self.d

    @property
    def n_tot(self) -> int:
        return (self.M + 1) * self.Nd

    def noisy(self, mu: np.ndarray) -> np.ndarray:
        """mu_eps = mu + noise_level * ||mu||_2 * noise."""
        mu = np.asarray(mu, dtype=np.float64)
        return mu + self.noise_level * float(np.linalg.norm(mu)) * self.noise


def grid_points(N: int, length: float) -> np.ndarray:
    return np.arange(1, N + 1, dtype=np.float64) * (length / (N + 1))


def time_points(M: int, T: float) -> np.ndarray:
    return np.arange(1, M + 1, dtype=np.float64) * (T / M)


def _mesh(d: int, N: int, length: float):
    x = grid_points(N, length)
    if d == 1:
        return (x,)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    return (X1.ravel(), X2.ravel())


def synthetic(d: int, N: int, M: int, beta: float, omega: float, alpha: float, *,
              T: float = 1.0, config_id: int = 0, instance: int = 0,
              amp1: float | None = 0.5, amp2: float | None = 0.3,
              modes: int = 5, noise_level: float = 1e-3, name: str = "synthetic") -> Inputs:
    """The smooth variable-coefficient family on the unit domain:
         gamma1 = 1 + a1 * prod(x) * t,  gamma2 = 1 + a2 * prod(sin(pi x)) * (1 + t),
         q = 1 + t, rho = 0,
         f = sum of sine modes with N(0,1)/|k|^2 coefficients (k in 1..modes per direction),
         Gaussian noise direction of unit 2-norm.
    amp1/amp2 = None draws the amplitude from U(0.1, 0.5)."""
    rng = np.random.default_rng([SEED_BASE, config_id, instance])
    a1 = float(rng.uniform(0.1, 0.5)) if amp1 is None else amp1
    a2 = float(rng.uniform(0.1, 0.5)) if amp2 is None else amp2
    X = _mesh(d, N, 1.0)
    t = time_points(M, T)
    px = np.prod(np.stack(X), axis=0)
    sx = np.prod(np.stack([np.sin(math.pi * xi) for xi in X]), axis=0)
    gamma1 = 1.0 + a1 * np.outer(t, px)
    gamma2 = 1.0 + a2 * np.outer(1.0 + t, sx)
    q = 1.0 + t
    Nd = N ** d
    rho = np.zeros(Nd)
    if d == 1:
        k = np.arange(1, modes + 1)
        c = rng.standard_normal(modes) / k ** 2
        f = np.sin(math.pi * np.outer(X[0], k)) @ c
    else:
        k1, k2 = np.meshgrid(np.arange(1, modes + 1), np.arange(1, modes + 1), indexing="ij")
        c = rng.standard_normal((modes, modes)) / (k1 ** 2 + k2 ** 2)
        S1 = np.sin(math.pi * np.outer(X[0], np.arange(1, modes + 1)))
        S2 = np.sin(math.pi * np.outer(X[1], np.arange(1, modes + 1)))
        f = np.einsum("pa,pb,ab->p", S1, S2, c)
    xi = rng.standard_normal(Nd)
    xi /= np.linalg.norm(xi)
    return Inputs(name=name, d=d, N=N, M=M, T=T, beta=beta, omega=omega, alpha=alpha,
                  length=1.0, gamma1=gamma1, gamma2=gamma2, q=q, rho=rho, f_true=f,
                  noise=xi, noise_level=noise_level)


def paper_problem(d: int, n: int, S: int, beta: float, omega: float, lam: float,
                  eps: float = 0.01, instance: int = 0) -> Inputs:
    """The paper's test problems of §6: Omega = (0, pi)^d, T = 1,
         d = 1: gamma1 = t e^x, gamma2 = t^2 x, q = t^2, rho = 0, f = x sin x;
         d = 2: gamma1 = t e^(x1+x2), gamma2 = t^2 x1 x2, q = t^2, rho = 0,
                f = x1 x2 sin(x1 x2);
    noise delta ~ U(-1, 1) pointwise, scaled by eps * ||mu||_2."""
    rng = np.random.default_rng([SEED_BASE, 100 + d, instance])
    X = _mesh(d, n, math.pi)
    t = time_points(S, 1.0)
    if d == 1:
        g1 = np.outer(t, np.exp(X[0]))
        g2 = np.outer(t ** 2, X[0])
        f = X[0] * np.sin(X[0])
    else:
        g1 = np.outer(t, np.exp(X[0] + X[1]))
        g2 = np.outer(t ** 2, X[0] * X[1])
        f = X[0] * X[1] * np.sin(X[0] * X[1])
    Nd = n ** d
    noise = rng.uniform(-1.0, 1.0, Nd)
    return Inputs(name=f"paper{d}d", d=d, N=n, M=S, T=1.0, beta=beta, omega=omega, alpha=lam,
                  length=math.pi, gamma1=g1, gamma2=g2, q=t ** 2, rho=np.zeros(Nd), f_true=f,
                  noise=noise, noise_level=eps)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def c1() -> Inputs:
    """d=1, N=63, M=32, beta=0.5, omega=1.5, alpha=1e-3, 5 sine modes (dense-parity size)."""
    return synthetic(1, 63, 32, 0.5, 1.5, 1e-3, config_id=1, modes=5, name="c1")


def c2(which: int = 0) -> Inputs:
    """d=1, N=4095, M=1024, (beta, omega) in {(0.3,1.2), (0.7,1.8)}, alpha=1e-4,
    amplitudes ~ U(0.1, 0.5), 20 sine modes."""
    beta, omega = [(0.3, 1.2), (0.7, 1.8)][which]
    return synthetic(1, 4095, 1024, beta, omega, 1e-4, config_id=2, instance=which,
                     amp1=None, amp2=None, modes=20, name=f"c2{'ab'[which]}")


def c3(instance: int = 0) -> Inputs:
    """d=2, N=255 per direction, M=256, beta=0.6, omega=1.6, alpha=1e-4, 8x8 sine modes; further
    instances draw other source modes and noise."""
    return synthetic(2, 255, 256, 0.6, 1.6, 1e-4, config_id=3, instance=instance, modes=8,
                     name="c3" if instance == 0 else f"c3_{instance}")


C4_SIZE = 64


def c4(instance: int) -> Inputs:
    """Instance k of the mixed batch of 64 (a stand-in for many independent problems): even k in
    d = 1 with N ~ U[127, 2047], odd k in d = 2 with N ~ U[31, 127]; M ~ U[64, 512],
    beta ~ U(0.2, 0.9), omega ~ U(1.1, 1.9), alpha log-uniform on [1e-5, 1e-2], coefficient
    amplitudes ~ U(0.1, 0.5)."""
    if not 0 <= instance < C4_SIZE:
        raise ValueError(f"c4 instance must be in [0, {C4_SIZE})")
    rng = np.random.default_rng([SEED_BASE, 4, 1000 + instance])
    d = 1 + instance % 2
    N = int(rng.integers(127, 2048)) if d == 1 else int(rng.integers(31, 128))
    M = int(rng.integers(64, 513))
    beta = float(rng.uniform(0.2, 0.9))
    omega = float(rng.uniform(1.1, 1.9))
    alpha = float(10.0 ** rng.uniform(-5.0, -2.0))
    return synthetic(d, N, M, beta, omega, alpha, config_id=4, instance=instance, amp1=None, amp2=None,
                     modes=min(8, N), name=f"c4_{instance}")


FIELD_K = 16  # control values per direction of the gradient workload's gamma2 field


def bilinear_weights(N: int, K: int = FIELD_K, length: float = 1.0) -> np.ndarray:
    """(N^2, K^2) weights of bilinear interpolation from a K x K grid of control values at
    xi_k = k length/(K-1), k = 0..K-1 per direction (row-major, last index fastest), to the interior
    grid points x_j = j length/(N+1) (last index fastest).  Each row has at most four nonzeros and
    sums to one."""
    x = grid_points(N, length) / length * (K - 1)
    i0 = np.clip(np.floor(x).astype(int), 0, K - 2)
    t = x - i0
    W1 = np.zeros((N, K))
    W1[np.arange(N), i0] = 1.0 - t
    W1[np.arange(N), i0 + 1] += t
    return np.kron(W1, W1)


def c5_field(instance: int = 0) -> np.ndarray:
    """The K x K control values of the gradient workload's gamma2 field, U(0.8, 1.2), from a
    generator of its own (the other draws of the instance are unchanged)."""
    rng = np.random.default_rng([SEED_BASE, 5, 100000 + instance])
    return rng.uniform(0.8, 1.2, size=(FIELD_K, FIELD_K))


def c5(instance: int = 0) -> Inputs:
    """The gradient workload's instance: d = 2, N = 127 per direction, M = 128, beta = 0.5,
    omega = 1.5, alpha = 1e-3, gamma1 amplitude ~ U(0.1, 0.5), 8 x 8 sine modes; gamma2 is the
    bilinear interpolation of a 16 x 16 field of control values ~ U(0.8, 1.2) (c5_field), the same at
    every time level."""
    inp = synthetic(2, 127, 128, 0.5, 1.5, 1e-3, config_id=5, instance=instance, amp1=None, amp2=None,
                    modes=8, name=f"c5_{instance}")
    g2 = bilinear_weights(inp.N) @ c5_field(instance).reshape(-1)
    return dataclasses.replace(inp, gamma2=np.tile(g2, (inp.M, 1)))


def small(d: int, N: int, M: int, beta: float = 0.5, omega: float = 1.5, alpha: float = 1e-3,
          instance: int = 0) -> Inputs:
    """A small instance of the same family for parity tests (seeded by its shape)."""
    return synthetic(d, N, M, beta, omega, alpha, config_id=1000 + 100 * d + N, instance=instance,
                     amp1=None, amp2=None, modes=min(5, N), name=f"small{d}d_{N}_{M}")
