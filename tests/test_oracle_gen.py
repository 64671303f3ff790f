"""Pins of the oracle's network generators: structural invariants, closed-form special
cases and distribution statistics (Sec. III-A.2 generator; ER by per-pair trials)."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from paper_1912_07423_amd import workloads as W


def _rows(net):
    rp = net.row_ptr().astype(np.int64)
    col = net.col()
    return [col[rp[i]:rp[i + 1]] for i in range(net.n)]


def test_er_structure_and_edge_count():
    spec = W.cuba_lif_4k(n_exc=800, n_inh=200, p=0.05)
    net = oracle.OracleNet(spec)
    n = net.n
    for i, r in enumerate(_rows(net)):
        assert np.all(np.diff(r) > 0)
        assert np.all((r >= 0) & (r < n)) and i not in set(r.tolist())
    mean = n * (n - 1) * 0.05
    sd = math.sqrt(n * (n - 1) * 0.05 * 0.95)
    assert abs(net.nnz - mean) < 5 * sd


def test_er_in_degree_binomial():
    spec = W.cuba_lif_4k(n_exc=800, n_inh=200, p=0.05)
    net = oracle.OracleNet(spec)
    indeg = np.bincount(net.col(), minlength=net.n)
    # each in-degree ~ Binomial(n-1, p); compare the histogram by chi-square
    n, p = net.n, 0.05
    lo, hi = int(n * p - 4 * math.sqrt(n * p)), int(n * p + 4 * math.sqrt(n * p))
    edges = np.arange(lo, hi + 1)
    obs = np.array([(indeg == k).sum() for k in edges])
    exp = np.array([scipy.stats.binom.pmf(k, n - 1, p) for k in edges]) * n
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-6, keep.sum())


def test_er_closed_forms_p0_p1():
    s0 = W.cuba_lif_4k(n_exc=40, n_inh=10, p=0.0)
    assert oracle.OracleNet(s0).nnz == 0
    s1 = W.cuba_lif_4k(n_exc=40, n_inh=10, p=1.0)
    net = oracle.OracleNet(s1)
    assert net.nnz == 50 * 49
    for i, r in enumerate(_rows(net)):
        assert list(r) == [j for j in range(50) if j != i]


def test_q16_weights_closed_form():
    net = oracle.OracleNet(W.cuba_lif_4k(n_exc=80, n_inh=20, p=0.2))
    rp = net.row_ptr().astype(np.int64)
    wq = net.w_q16()
    # round-half-even(w * 2^16): 0.27 mV -> 17695 (17694.72), -4.5 mV -> -294912
    assert set(wq[: rp[80]].tolist()) == {17695}
    assert set(wq[rp[80]:].tolist()) == {-294912}
    b = oracle.OracleNet(W.brunel_fixed_out(n=500, k=20, delay_steps=2, n_ext=0))
    rp = b.row_ptr().astype(np.int64)
    assert set(b.w_q16()[: rp[400]].tolist()) == {6554}      # 0.1 mV -> 6553.6
    assert set(b.w_q16()[rp[400]:].tolist()) == {-32768}     # -0.5 mV


def test_fixed_out_structure():
    spec = W.brunel_fixed_out(n=1000, k=37, delay_steps=3, n_ext=0)
    net = oracle.OracleNet(spec)
    assert net.nnz == 1000 * 37
    for i, r in enumerate(_rows(net)):
        assert len(r) == 37 and np.all(np.diff(r) > 0)
        assert r[0] >= 0 and r[-1] < 1000 and i not in set(r.tolist())


def test_fixed_out_closed_forms():
    # k = all candidates: every other neuron; k = 0: no edges
    net = oracle.OracleNet(W.brunel_fixed_out(n=50, k=49, delay_steps=1, n_ext=0))
    for i, r in enumerate(_rows(net)):
        assert list(r) == [j for j in range(50) if j != i]
    assert oracle.OracleNet(W.brunel_fixed_out(n=50, k=0, delay_steps=1, n_ext=0)).nnz == 0


def _spacing_values(n, k, seeds):
    """e_k = x_k - k of every row (Fig. 2 (e)), per row."""
    spec = W.brunel_fixed_out(n=n, k=k, delay_steps=1, n_ext=0)
    out = []
    for seed in seeds:
        spec["params"]["seed"] = seed
        net = oracle.OracleNet(spec)
        for i, r in enumerate(_rows(net)):
            local = r - (r > i)            # candidate index in [0, n-1)
            out.append(local - np.arange(k))
    return np.array(out)


def _bin_probs(m):
    """round-half-up(U * m) for U ~ U(0,1): half-width bins at 0 and m."""
    p = np.full(m + 1, 1.0 / m)
    p[0] = p[-1] = 0.5 / m
    return p


def test_fixed_out_scaled_values_are_rounded_uniforms():
    """Fig. 2 (c)-(e): the exponential spacings normalised by their total are the order
    statistics of k i.i.d. U(0,1); scaled by the spare count m = M - k and rounded,
    the values e_k = x_k - k are k sorted i.i.d. draws with P(0) = P(m) = 1/(2m) and
    P(v) = 1/m inside.  Pins the exclusive scan, the normalisation, the scale b-a-n,
    the rounding and the +k step at once."""
    n, k = 400, 40
    e = _spacing_values(n, k, range(100, 106))
    m = (n - 1) - k
    assert e.min() >= 0 and e.max() <= m and np.all(np.diff(e, axis=1) >= 0)
    obs = np.bincount(e.ravel(), minlength=m + 1)
    exp = _bin_probs(m) * e.size
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-6, m)


def test_fixed_out_endpoints_reachable_not_forced():
    """With the sentinels the first and last candidates are selected with probability
    1 - (1 - 1/(2m))^k each (e_1 = 0, resp. e_k = m), not always."""
    n, k = 400, 40
    e = _spacing_values(n, k, range(200, 206))
    m = (n - 1) - k
    p_end = 1 - (1 - 0.5 / m) ** k
    rows = e.shape[0]
    sd = math.sqrt(rows * p_end * (1 - p_end))
    assert abs((e[:, 0] == 0).sum() - rows * p_end) < 5 * sd
    assert abs((e[:, -1] == m).sum() - rows * p_end) < 5 * sd
    assert 0 < (e[:, 0] == 0).sum() < rows


def test_fixed_out_ties_of_iid_draws():
    """Adjacent candidates are both selected exactly when e_{k+1} = e_k; for k i.i.d.
    draws the expected number of such ties is k - sum_v (1 - (1 - p_v)^k)."""
    n, k = 200, 50
    e = _spacing_values(n, k, range(7, 12))
    m = (n - 1) - k
    pv = _bin_probs(m)
    exp_ties = k - np.sum(1 - (1 - pv) ** k)
    ties = (np.diff(e, axis=1) == 0).sum(axis=1)
    assert abs(ties.mean() - exp_ties) < 5 * ties.std() / math.sqrt(len(ties))


@pytest.mark.parametrize("make", [
    lambda: W.cuba_lif_4k(n_exc=160, n_inh=40, p=0.1),
    lambda: W.brunel_fixed_out(n=300, k=25, delay_steps=4, n_ext=0),
    lambda: W.stdp_er(n=250, p=0.1, n_ext=0),
])
def test_gen_row_equals_built_rows(make):
    spec = make()
    net = oracle.OracleNet(spec)
    rows = _rows(net)
    for i in [0, 1, net.n // 2, net.n - 1]:
        col, _, _ = oracle.gen_row(spec, i)
        assert np.array_equal(col, rows[i])


def test_invalid_specs_rejected():
    bad = W.brunel_fixed_out(n=50, k=50, delay_steps=1, n_ext=0)   # k > n-1 candidates
    with pytest.raises(ValueError):
        oracle.OracleNet(bad)
    bad = W.cuba_lif_4k(n_exc=10, n_inh=10, p=1.5)
    with pytest.raises(ValueError):
        oracle.OracleNet(bad)
    bad = W.cuba_lif_4k(n_exc=10, n_inh=10)
    bad["params"]["delay_steps"] = 0
    with pytest.raises(ValueError):
        oracle.OracleNet(bad)
