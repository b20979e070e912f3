"""SFH and enrichment history -> SSP weights W_ma, step scheme (Sec. 2.2, App. B).

Per parameter vector:
  * lookback edges T_0 = 0 < T_1 < ... < T_{N_T}; the grid is rescaled to the age
    of the Universe at the sampled redshift (Sec. 2.6): T_1 fixed, T_1..T_{N_T}
    log-uniform up to t_univ(z).  Bin masses m_i are parameters, so the formed
    mass is unchanged by the rescaling (Sec. 2.2.1).
  * step scheme (App. B, the FastStepBasis convention): the SFR is constant in
    each bin and the bin's mass goes to the SSP age nodes in proportion to the
    linear-time overlap between the bin and each node's cell, the cell being
    bounded by the midpoints to its neighbours.  Reading: the first cell starts
    at 0 and the last one extends to +infinity, so every bin's mass is assigned.
  * each bin's mass is split between the two bracketing metallicity nodes by
    linear interpolation in log10(Z/Zsun) (Sec. 2.2.2, App. B), and likewise on
    an [alpha/Fe] axis when the library has one (Sec. 5.4).
"""
import numpy as np


def sfh_edges(t_univ, n_sfh, T1):
    """Edges [n_sfh+1]: 0, then n_sfh values log-uniform from T1 to t_univ (inclusive)."""
    if not t_univ > T1:
        raise ValueError("age of the Universe must exceed the first SFH edge")
    return np.concatenate([[0.0], np.geomspace(T1, t_univ, n_sfh)])


def age_cells(ages):
    """Linear-time Voronoi cells of the SSP age nodes: lo_0 = 0, hi_last = +inf."""
    ages = np.asarray(ages, dtype=np.float64)
    mid = 0.5 * (ages[:-1] + ages[1:])
    lo = np.concatenate([[0.0], mid])
    hi = np.concatenate([mid, [np.inf]])
    return lo, hi


def step_weights(edges, masses, lo, hi):
    """w[i, a] = m_i * |[T_i, T_{i+1}] intersect [lo_a, hi_a]| / (T_{i+1} - T_i)."""
    Ti = edges[:-1, None]
    Tj = edges[1:, None]
    overlap = np.minimum(hi[None, :], Tj) - np.maximum(lo[None, :], Ti)
    overlap = np.maximum(overlap, 0.0)
    return masses[:, None] * overlap / (Tj - Ti)


def bin_metallicity_hist(zh_nodes, edges, T1, t_univ):
    """Per-bin metallicity of the time-varying mode (Sec. 2.2.2).

    Reading: the N_ZH enrichment nodes sit log-uniformly from T1 to t_univ(z),
    rescaled with the SFH grid; bin i takes the value interpolated linearly in
    ln T at its centre (geometric mean of its edges; the first bin, which starts
    at T=0, uses T1/2), clamped to the end nodes.
    """
    n_zh = len(zh_nodes)
    node_t = np.geomspace(T1, t_univ, n_zh)
    centres = np.empty(len(edges) - 1)
    centres[0] = 0.5 * T1
    centres[1:] = np.sqrt(edges[1:-1] * edges[2:])
    return np.interp(np.log(centres), np.log(node_t), zh_nodes)


def grid_split(x, nodes):
    """Bracketing node j and fraction t of x on a 1-D grid (clamped to the grid).

    j = max{j : nodes_j <= x} limited to [0, N-2]; t = (x - nodes_j)/(nodes_{j+1} - nodes_j),
    so x on the last node gives (N-2, 1) and x below the first gives (0, 0).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    xc = min(max(float(x), nodes[0]), nodes[-1])
    j = int(np.searchsorted(nodes, xc, side="right")) - 1
    j = min(max(j, 0), len(nodes) - 2)
    t = (xc - nodes[j]) / (nodes[j + 1] - nodes[j])
    return j, t


def ssp_weights(w, zeta, logz_nodes, afe=0.0, afe_nodes=(0.0,)):
    """W[alpha, m, a]: mass formed at each SSP node (eq. 1, eq. B1)."""
    n_z = len(logz_nodes)
    n_af = len(afe_nodes)
    W = np.zeros((n_af, n_z, w.shape[1]))
    if n_af > 1:
        ja, ta = grid_split(afe, afe_nodes)
        asplit = ((ja, 1.0 - ta), (ja + 1, ta))
    else:
        asplit = ((0, 1.0),)
    for i in range(w.shape[0]):
        if n_z > 1:
            jz, tz = grid_split(zeta[i], logz_nodes)
            zsplit = ((jz, 1.0 - tz), (jz + 1, tz))
        else:
            zsplit = ((0, 1.0),)
        for ia, fa in asplit:
            for iz, fz in zsplit:
                W[ia, iz, :] += fa * fz * w[i, :]
    return W
