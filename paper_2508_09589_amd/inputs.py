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


# ---------------------------------------------------------------------------
# The paper's two example problems (§2.3), in rescaled units (§2.1: L = 1,
# Delta T = 1, time rescaled by tau so that t~ runs over [0, 1], k~ = k tau,
# Q~ as printed).  Sizes are the caller's; the paper solves them at 640^2 x 1280
# and above.

# Default SIMP endpoints and penalties of §2.2 (physical units).
PAPER_MATERIAL = dict(k_ins=0.03, k_con=3.0, p_k=3.0, c_ins=0.5, c_con=1.0, p_c=2.0)

# Material variants of §5.1.3 and §5.2.2: B = defaults, C/D = more conductive
# or more capacitive conductive phase.  Example 1D also raises p_c to 4.
EXAMPLE_VARIANTS = {
    "1B": dict(example=1),
    "1C": dict(example=1, k_con=10.0),
    "1D": dict(example=1, c_con=100.0, p_c=4.0),
    "2B": dict(example=2),
    "2C": dict(example=2, c_con=100.0),
}
EXAMPLE_TAU = {1: 1.0, 2: 6.0}
# Example 1: heat sink of width L/10 at the centre of the lower edge (x2 = 0).
# Example 2: every outer wall is cold.
EXAMPLE_PATCHES = {1: ((2, 0.5, 0.05),),
                   2: ((0, 0.5, 0.5), (1, 0.5, 0.5), (2, 0.5, 0.5), (3, 0.5, 0.5))}


def example1_source(n, nt, q0=100.0):
    """Nodal Q~ of Example 1 [nt+1, n+1, n+1]: uniform in space, in time
    q0/2 (1 - t)(1 + cos 50 t) on t in [0, 1] (tau = 1)."""
    t = np.arange(nt + 1) / nt
    q = 0.5 * q0 * (1.0 - t) * (1.0 + np.cos(50.0 * t))
    return np.broadcast_to(q[:, None, None], (nt + 1, n + 1, n + 1)).copy()


def example2_centre(t):
    """Centre of the Example 2 source at physical time t (R = 0.25, omega =
    pi, starting at (L/2, 3L/4))."""
    a = np.pi * np.asarray(t, dtype=np.float64) + 0.5 * np.pi
    return 0.5 + 0.25 * np.cos(a), 0.5 + 0.25 * np.sin(a)


def example2_source(n, nt, q0=1.0, sigma=0.05):
    """Nodal Q~ of Example 2 [nt+1, n+1, n+1]: a Gaussian of peak q0 and width
    sigma whose centre circles the domain centre; rescaled time t~ = t / 6
    (three rotations)."""
    t = 6.0 * np.arange(nt + 1) / nt
    c1, c2 = example2_centre(t)
    x = np.arange(n + 1) / n
    d1 = (x[None, None, :] - c1[:, None, None]) ** 2          # x1 varies along the last axis
    d2 = (x[None, :, None] - c2[:, None, None]) ** 2          # x2 along the middle one
    return q0 * np.exp(-(d1 + d2) / (2.0 * sigma * sigma))


def example_problem(variant, n, nt):
    """Keyword arguments of one example variant at an n^2 x nt grid: rescaled
    material (k~ = k tau), patches, nodal source, dx = 1/n, dt = 1/nt."""
    v = dict(EXAMPLE_VARIANTS[variant])
    ex = v.pop("example")
    mat = dict(PAPER_MATERIAL, **v)
    tau = EXAMPLE_TAU[ex]
    mat["k_ins"] *= tau
    mat["k_con"] *= tau
    src = example1_source(n, nt) if ex == 1 else example2_source(n, nt)
    return dict(nx=n, ny=n, nt=nt, dx=1.0 / n, dt=1.0 / nt, patches=EXAMPLE_PATCHES[ex],
                source=src, **mat)


def example_design(kind, n):
    """Time-constant designs [n, n] for the example comparisons: "uniform" =
    0.3 everywhere (a volume-fraction start); "tree" = a binary conductive
    tree (rho 1 / 0.001 at element centres) whose trunk leaves the lower edge
    at x1 = 0.5 and reaches x2 = 0.9, with eight branches across it; trunk and
    branches are at least one element wide at any n."""
    if kind == "uniform":
        return np.full((n, n), 0.3)
    if kind != "tree":
        raise KeyError(kind)
    c = (np.arange(n) + 0.5) / n
    x2, x1 = np.meshgrid(c, c, indexing="ij")      # [ny, nx]
    hw_t, hw_b = max(0.03, 0.5 / n), max(0.018, 0.5 / n)
    solid = (x2 <= 0.9) & (np.abs(x1 - 0.5) <= hw_t)
    for k in range(1, 9):
        solid |= (np.abs(x2 - 0.1 * k) <= hw_b) & (x1 >= 0.05) & (x1 <= 0.95)
    return np.where(solid, 1.0, 0.001)
