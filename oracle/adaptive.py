"""Sketch size from the effective dimension, and reuse of the preconditioner
across IP-PMM iterations (section "Convergence analysis of Nys-IP-PMM":
the main theorem with eq. main-thm-sketch-size; eq. effective-dim; the
closing remark of the rank study in section 5, which names tuning the rank
per problem and reusing the preconditioner between iterations as the next
improvements).

Definitions followed:
* d_eff(N, mu) = tr(N (N + mu I)^{-1}) = sum_i lambda_i / (lambda_i + mu)
  (eq. effective-dim).
* The theorem's sketch size at IP-PMM iteration k:
  ell_k >= 8 (sqrt(d_eff(N_k, mu_k)) + sqrt(32 log(16 (k + 2))))^2, with the
  natural logarithm.

Readings (the paper states the bound but no practical rule, and no rule for
reuse):
* d_eff(N_k, mu_k) is estimated from the eigenvalues lambda_hat (descending)
  of the most recent Nystrom approximation, taken at the current mu_k:
  d_hat = sum_i lambda_hat_i / (lambda_hat_i + mu_k).  The Nystrom
  approximation satisfies N_hat <= N in the Loewner order, so
  lambda_hat_i <= lambda_i and d_hat <= d_eff(N, mu) when both are taken for
  the same N.
* Rule "deff": target = ceil(c_ell d_hat); when lambda_hat_ell > mu_k the
  previous sketch saw no eigenvalue below mu_k, so d_eff may lie beyond its
  reach and target = max(target, 2 ell_prev); ell_k = min(ell_max,
  max(ell_min, target)).
* Rule "theorem": target = ceil(8 (sqrt(d_hat) + sqrt(32 log(16 (k+2))))^2),
  clamped to [ell_min, ell_max] (the bound itself is at least 887).
* Reuse with maximal age a and growth factor g: build at the first IP-PMM
  iteration; afterwards rebuild at iteration k when k - k_build >= a, or when
  the PCG iterations of iteration k-1 (predictor plus corrector) exceed g
  times those of iteration k_build.  Otherwise the previous (U, lambda_hat)
  are kept and applied with the current delta_k (eq. Nys_precond_inv), or
  the previous partial Cholesky factor is kept.

Test infrastructure (see the package docstring).
"""

import math

import numpy as np

RULE_FIXED, RULE_DEFF, RULE_THEOREM = 0, 1, 2


def d_eff(eigs, mu):
    """eq. effective-dim from the eigenvalues of N (negative rounding noise
    counted as 0)."""
    lam = np.clip(np.asarray(eigs, dtype=np.float64), 0.0, None)
    return float(np.sum(lam / (lam + mu)))


def d_eff_matrix(N, mu):
    """d_eff of a symmetric positive semidefinite matrix, through its
    eigenvalues."""
    return d_eff(np.linalg.eigvalsh(np.asarray(N, dtype=np.float64)), mu)


def d_eff_estimate(lam_hat, mu):
    """Estimate of d_eff(N, mu) from the Nystrom eigenvalues lambda_hat."""
    return d_eff(lam_hat, mu)


def theorem_sketch_size(deff, k):
    """Right-hand side of eq. main-thm-sketch-size at IP-PMM iteration k."""
    return 8.0 * (math.sqrt(deff) + math.sqrt(32.0 * math.log(16.0 * (k + 2)))) ** 2


def sketch_size_rule(rule, d_hat, lam_last, mu, k, ell_prev, ell_min, ell_max, c_ell):
    """Sketch size for the preconditioner built at IP-PMM iteration k."""
    if rule == RULE_FIXED:
        return int(ell_prev)
    if rule == RULE_DEFF:
        target = math.ceil(c_ell * d_hat)
        if lam_last > mu:
            target = max(target, 2 * ell_prev)
    elif rule == RULE_THEOREM:
        target = math.ceil(theorem_sketch_size(d_hat, k))
    else:
        raise ValueError(f"unknown sketch-size rule {rule}")
    return int(min(ell_max, max(ell_min, target)))


def rebuild_due(k, k_build, pcg_prev, pcg_ref, max_age, growth):
    """True when the preconditioner is built anew at IP-PMM iteration k.
    k_build < 0: none built yet.  max_age <= 0: no reuse (build every
    iteration)."""
    if k_build < 0 or max_age <= 0:
        return True
    if k - k_build >= max_age:
        return True
    return pcg_prev > growth * pcg_ref
