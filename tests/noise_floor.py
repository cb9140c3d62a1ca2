"""Closed-form sampling noise of the cumulant norms of Gaussian windows
(a statistical pin for the norms of Alg. 5 and Eq. (mef), independent of
how either side computes them)."""
import numpy as np


def gaussian_noise_floor(S, t, k):
    """Leading-order E ||C_k-hat||_F^2 for t i.i.d. N(mu, S) rows, k = 3, 4.
    Under Gaussianity the sample k-th cumulant tensor has zero mean and
    covariance (1/t) sum over the bijections sigma between the two index
    sets of prod_m S[i_m, j_sigma(m)] (the normal-theory variance of
    k-statistics); summing its diagonal over all n^k positions leaves, per
    sigma, the product over the cycles of sigma of tr(S^|cycle|): the cycle
    index of the symmetric group S_k."""
    tr = lambda e: float(np.trace(np.linalg.matrix_power(S, e)))
    if k == 3:  # S_3: 1 identity, 3 transpositions, 2 three-cycles
        return (tr(1) ** 3 + 3 * tr(2) * tr(1) + 2 * tr(3)) / t
    # S_4: 1 identity, 6 transpositions, 3 double transpositions,
    # 8 three-cycles, 6 four-cycles
    return (tr(1) ** 4 + 6 * tr(2) * tr(1) ** 2 + 3 * tr(2) ** 2 + 8 * tr(3) * tr(1) + 6 * tr(4)) / t
