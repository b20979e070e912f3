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


def _log_moments(X):
    """A = int_0^X ln(1+x) dx and B = int_0^X x ln(1+x) dx, by their closed forms, or by
    their Taylor series below X = 0.05 (where the closed forms cancel)."""
    if X < 0.05:
        A = sum((-1) ** k * X ** k / (k * (k - 1)) for k in range(2, 16))
        B = sum((-1) ** (n + 1) * X ** (n + 2) / (n * (n + 2)) for n in range(1, 15))
        return A, B
    lp = np.log1p(X)
    return (1.0 + X) * lp - X, 0.5 * (X * X - 1.0) * lp - 0.25 * X * X + 0.5 * X


def _piece(psi_u, beta, u, v):
    """For psi(t) = psi_u + beta (t - u) on [u, v]: (int psi dt, int psi ln(t/u) dt), written
    about the piece's own lower end so that no large terms cancel."""
    X = (v - u) / u
    A, B = _log_moments(X)
    return (v - u) * (psi_u + 0.5 * beta * (v - u)), u * (psi_u * A + beta * u * B)


def tent_weights(edges, psi_nodes, ages):
    """Linear scheme (App. B, eq. tent_integral): w[i, a], the mass of SFH bin i given to
    SSP age node a.

    The SFR is piecewise linear in lookback time through (T_i, psi_i); the spectrum between
    adjacent age nodes t_j < t_{j+1} is the linear-in-ln t mix a_j(t) s(t_j) + b_{j+1}(t)
    s(t_{j+1}), a_j = ln(t_{j+1}/t) / ln(t_{j+1}/t_j), b_{j+1} = 1 - a_j, so node j takes
    int psi a_j over [t_j, t_{j+1}] plus int psi b_j over [t_{j-1}, t_j], each split at the
    bin edges and evaluated in closed form, written about each piece's lower end u (the
    SFR as psi(u) + beta (t - u), ln t as ln u + ln(1 + (t - u)/u)) so that no large terms
    cancel: the naive form alpha + beta t, alpha = psi_i - beta T_i, loses up to ~1e-11.
    Each bin's weights are clipped at zero and rescaled to its trapezoidal mass
    (psi_i + psi_{i+1}) (T_{i+1} - T_i) / 2.

    Readings: psi_nodes holds psi at T_0 .. T_{n-1} (n = number of bins, element 0 the
    most recent) and the SFR at the oldest edge T_n repeats psi_{n-1}; lookback times
    below the youngest age node or above the oldest belong to that end node alone (the
    interpolation is clamped, like the metallicity axis).
    """
    edges = np.asarray(edges, dtype=np.float64)
    n = len(edges) - 1
    psi = np.concatenate([np.asarray(psi_nodes, dtype=np.float64), [psi_nodes[-1]]])
    t = np.asarray(ages, dtype=np.float64)
    na = len(t)
    w = np.zeros((n, na))
    for i in range(n):
        T0, T1 = edges[i], edges[i + 1]
        beta = (psi[i + 1] - psi[i]) / (T1 - T0)
        at = lambda x: psi[i] + beta * (x - T0)            # the SFR at x in the bin
        # below the youngest node: all to node 0
        u, v = T0, min(T1, t[0])
        if v > u:
            w[i, 0] += (v - u) * (at(u) + 0.5 * beta * (v - u))
        # between nodes j and j+1: node j takes int psi ln(t_{j+1}/t), node j+1 int psi
        # ln(t/t_j), each over ln(t_{j+1}/t_j); with I = int psi ln(t/u) about the piece's
        # lower end u: ln(t_{j+1}/u) int psi - I and ln(u/t_j) int psi + I
        for j in range(na - 1):
            u, v = max(T0, t[j]), min(T1, t[j + 1])
            if v <= u:
                continue
            i0, I = _piece(at(u), beta, u, v)
            dL = np.log(t[j + 1] / t[j])
            w[i, j] += (np.log(t[j + 1] / u) * i0 - I) / dL
            w[i, j + 1] += (np.log(u / t[j]) * i0 + I) / dL
        # above the oldest node: all to the last node
        u, v = max(T0, t[-1]), T1
        if v > u:
            w[i, -1] += (v - u) * (at(u) + 0.5 * beta * (v - u))
        w[i] = np.maximum(w[i], 0.0)
        m_i = 0.5 * (psi[i] + psi[i + 1]) * (T1 - T0)
        s = w[i].sum()
        if s > 0.0:
            w[i] *= m_i / s
    return w
