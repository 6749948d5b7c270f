"""Seeded synthetic inputs for the space-time heat-conduction workloads.

This module only draws and shapes input data (densities, patches, request
streams).  It holds none of the solver's arithmetic, so both the GPU path and
the FP64 oracle may take their inputs from it.

Workloads (all: unit square, tau = 1, T(0) = 0, uniform Q = 1, C = 1,
k = 1e-3 + (1 - 1e-3) rho^3, T = 0 on the centred 10% of the x1 = 0 edge):
  small      32^2  x 32,   time-constant rho ~ U[0.001, 1]          (seed 0)
  medium     256^2 x 256,  time-varying smooth field, corr. length 0.1 (seed 1)
  large      512^2 x 1024, time-constant heat-sink pattern, rho in {0.001, 1}
  grad       128^2 x 128,  time-varying smooth field (seed 2), filter r = 1.5 el.
  serving    256 requests, Poisson arrivals at 50/s (seed 4)
"""
import numpy as np

K_INS, K_CON, P_K = 1e-3, 1.0, 3.0
C_INS, C_CON, P_C = 1.0, 1.0, 1.0
PATCH_LEFT_CENTRED = (0, 0.5, 0.05)   # (edge x1 = 0, centre 0.5, half width 0.05)


def uniform_density(n, seed=0):
    """Time-constant density [n, n] drawn uniformly from [0.001, 1]."""
    return np.random.default_rng(seed).uniform(0.001, 1.0, (n, n))


def smooth_density(nx, ny, nt, seed=1, corr=0.1):
    """Time-varying density [nt, ny, nx]: Gaussian-correlated noise mapped to
    [0.001, 1] through the normal CDF (so its marginal is uniform).

    White noise N(0,1) per element is smoothed with a Gaussian kernel of
    standard deviation corr/sqrt(2) in unit-cube coordinates (covariance
    exp(-r^2 / (2 corr^2))), reflecting boundaries, then standardised."""
    from scipy.ndimage import gaussian_filter
    from scipy.special import ndtr
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nt, ny, nx))
    sig = corr / np.sqrt(2.0)
    z = gaussian_filter(z, sigma=(sig * nt, sig * ny, sig * nx), mode="reflect")
    z = (z - z.mean()) / z.std()
    return 0.001 + 0.999 * ndtr(z)


def heat_sink_density(n):
    """Time-constant heat-sink pattern [n, n]: a trunk along x2 = 0.5 from the
    sink edge and eight fingers across it; rho = 1 inside, 0.001 outside,
    tested at element centres (volume fraction about 0.3)."""
    c = (np.arange(n) + 0.5) / n
    x2, x1 = np.meshgrid(c, c, indexing="ij")      # [ny, nx]
    solid = (x1 <= 0.9) & (np.abs(x2 - 0.5) <= 0.03)
    for k in range(1, 9):
        solid |= (np.abs(x1 - 0.1 * k) <= 0.018) & (x2 >= 0.05) & (x2 <= 0.95)
    return np.where(solid, 1.0, 0.001)


WORKLOADS = {
    "small": dict(nx=32, ny=32, nt=32, time_varying=False),
    "medium": dict(nx=256, ny=256, nt=256, time_varying=True),
    "large": dict(nx=512, ny=512, nt=1024, time_varying=False),
    "grad": dict(nx=128, ny=128, nt=128, time_varying=True),
}


def workload_density(name):
    w = WORKLOADS[name]
    if name == "small":
        return uniform_density(32, seed=0)
    if name == "medium":
        return smooth_density(256, 256, 256, seed=1)
    if name == "large":
        return heat_sink_density(512)
    if name == "grad":
        return smooth_density(128, 128, 128, seed=2)
    raise KeyError(name)


def serving_requests(n_requests=256, rate=50.0, seed=4,
                     sizes=(32, 64, 128, 256), slabs=(32, 64, 128, 256)):
    """Request stream: exponential inter-arrival times (mean 1/rate s), square
    spatial grid n ~ U(sizes), nt ~ U(slabs), exactly half forward-only and half
    forward+adjoint (a random permutation); density seed = 1000*seed + id."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    n = rng.choice(sizes, n_requests)
    nt = rng.choice(slabs, n_requests)
    adj = np.zeros(n_requests, dtype=bool)
    adj[rng.permutation(n_requests)[: n_requests // 2]] = True
    return [dict(id=i, t_arrive=float(t[i]), n=int(n[i]), nt=int(nt[i]),
                 adjoint=bool(adj[i]), seed=1000 * seed + i) for i in range(n_requests)]
