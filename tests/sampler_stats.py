"""Statistics for checking Monte Carlo samples of the 4x4 lattice against the
exact distribution |psi|^2 / Z over all of its Sz = 0 states (no arithmetic
of the method here: the probabilities come in as an argument).

Three checks on independent samples (one per chain):
* the total variation distance between the histogram over every state and
  the exact distribution, against the same distance for multinomial draws
  from the exact distribution (a seeded simulation of its null spread);
* chi-square over 64 bins of equal exact mass, the states ordered by
  probability (a bias between likely and unlikely states);
* chi-square over 64 groups of a seeded random partition of the states (a
  bias that ignores probability, e.g. between states of equal
  magnetisation)."""
import numpy as np

NBINS = 64


def state_index(samples, states):
    """Row index in `states` (increasing bitmask order) of every sample."""
    N = states.shape[1]
    w = (np.int64(1) << np.arange(N, dtype=np.int64))
    ms = ((states > 0).astype(np.int64) * w).sum(axis=1)
    mq = ((samples > 0).astype(np.int64) * w).sum(axis=1)
    idx = np.searchsorted(ms, mq)
    assert (ms[idx] == mq).all(), "a sample is not an Sz = 0 state"
    return idx


def _chi2(counts, expected):
    return float((((counts - expected) ** 2) / expected).sum())


def check_histogram(samples, states, p, seed=2024, null_draws=300):
    """Returns a dict of the statistics and their bounds; asserts all three."""
    n = samples.shape[0]
    counts = np.bincount(state_index(samples, states), minlength=states.shape[0]).astype(np.float64)
    tv = 0.5 * np.abs(counts / n - p).sum()
    rng = np.random.default_rng(seed)
    null = np.array([0.5 * np.abs(rng.multinomial(n, p) / n - p).sum() for _ in range(null_draws)])
    tv_bound = null.mean() + 6 * null.std()
    # equal-mass bins of the states ordered by probability
    order = np.argsort(p, kind="stable")
    cum = np.cumsum(p[order])
    bin_of = np.minimum((cum * NBINS).astype(np.int64), NBINS - 1)
    b_counts = np.bincount(bin_of, weights=counts[order], minlength=NBINS)
    b_exp = np.bincount(bin_of, weights=p[order], minlength=NBINS) * n
    # a seeded random partition into NBINS groups
    grp = np.random.default_rng(seed + 1).integers(0, NBINS, size=states.shape[0])
    g_counts = np.bincount(grp, weights=counts, minlength=NBINS)
    g_exp = np.bincount(grp, weights=p, minlength=NBINS) * n
    dof = NBINS - 1
    chi_bound = dof + 6 * np.sqrt(2 * dof)
    out = dict(n=n, tv=tv, tv_null_mean=float(null.mean()), tv_bound=float(tv_bound),
               chi2_mass_bins=_chi2(b_counts, b_exp), chi2_random_groups=_chi2(g_counts, g_exp),
               chi2_bound=float(chi_bound))
    assert tv <= tv_bound, out
    assert out["chi2_mass_bins"] <= chi_bound, out
    assert out["chi2_random_groups"] <= chi_bound, out
    return out
