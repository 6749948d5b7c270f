"""Semi-coarsening level choice, Algorithm 1 of the paper (oracle).

The effective diffusivity D_eff = sqrt(k_con k_ins / (C_con C_ins)) is formed
once; on each level the anisotropy lambda = D_eff * dt / dx^2 decides: below
lambda_crit the next level halves the time resolution, otherwise it halves both
spatial resolutions (§3.2.1).

Full space-time coarsening (the comparison the paper makes in §5.1.2, drawn
beside the two semi-coarsenings in §3.2.1) halves all three resolutions on
every level.

Readings where the paper is silent:
  * the comparison is strict ("<"), so lambda == lambda_crit coarsens in space;
  * when the chosen direction cannot be halved (odd or unit element count) the
    other direction is tried, and when neither can the hierarchy stops;
  * the number of levels N_l is a user choice in the paper (8 for its
    space-time runs in §4, 7 in §5); max_levels defaults to 8, and the
    hierarchy also stops once a level has at most max_coarse_nodes nodes;
  * past max_levels coarsening continues only while the coarsest level is too
    large to be factorised exactly by the solver (planes of more than
    max_plane nodes, or a block factorisation of more than max_factor_bytes).
"""
import math

SPACE, TIME, FULL = "space", "time", "full"


def d_eff(k_con, k_ins, c_con, c_ins):
    return math.sqrt(k_con * k_ins / (c_con * c_ins))


def _can_halve_space(nx, ny):
    return nx % 2 == 0 and ny % 2 == 0 and nx >= 2 and ny >= 2


def _can_halve_time(nt):
    return nt % 2 == 0 and nt >= 2


def _factorable(L, max_plane, max_factor_bytes):
    P = (L["nx"] + 1) * (L["ny"] + 1)
    return P <= max_plane and P * P * 16.0 * (L["nt"] + 1) <= max_factor_bytes


def build_hierarchy(nx, ny, nt, dx, dt, k_con, k_ins, c_con, c_ins,
                    lambda_crit=0.5, n_levels=None, max_coarse_nodes=4096, max_levels=8,
                    full=False, max_plane=2048, max_factor_bytes=16.0 * 2 ** 30):
    """Return a list of dicts, one per level (finest first), with keys
    nx, ny, nt, dx, dt, lam (anisotropy of that level) and how (how the level
    was made from the one above it: None, 'space', 'time' or 'full').
    full=True: full space-time coarsening while all three counts can be
    halved (reading: the hierarchy stops when one of them cannot)."""
    D = d_eff(k_con, k_ins, c_con, c_ins)
    levels = [dict(nx=nx, ny=ny, nt=nt, dx=dx, dt=dt, how=None)]
    limit = n_levels if n_levels is not None else max_levels
    while len(levels) < (limit if n_levels is not None else 32):
        L = levels[-1]
        L["lam"] = D * L["dt"] / L["dx"] ** 2
        if n_levels is None and (L["nx"] + 1) * (L["ny"] + 1) * (L["nt"] + 1) <= max_coarse_nodes:
            break
        if n_levels is None and len(levels) >= limit and (
                max_levels < 2 or _factorable(L, max_plane, max_factor_bytes)):
            break
        if full:
            if not (_can_halve_space(L["nx"], L["ny"]) and _can_halve_time(L["nt"])):
                break
            levels.append(dict(nx=L["nx"] // 2, ny=L["ny"] // 2, nt=L["nt"] // 2,
                               dx=2 * L["dx"], dt=2 * L["dt"], how=FULL))
            continue
        want = TIME if L["lam"] < lambda_crit else SPACE
        order = (want, SPACE if want == TIME else TIME)
        how = None
        for d in order:
            if d == SPACE and _can_halve_space(L["nx"], L["ny"]):
                how = SPACE
                break
            if d == TIME and _can_halve_time(L["nt"]):
                how = TIME
                break
        if how is None:
            break
        if how == SPACE:
            levels.append(dict(nx=L["nx"] // 2, ny=L["ny"] // 2, nt=L["nt"],
                               dx=2 * L["dx"], dt=L["dt"], how=SPACE))
        else:
            levels.append(dict(nx=L["nx"], ny=L["ny"], nt=L["nt"] // 2,
                               dx=L["dx"], dt=2 * L["dt"], how=TIME))
    levels[-1]["lam"] = D * levels[-1]["dt"] / levels[-1]["dx"] ** 2
    return levels
