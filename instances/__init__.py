"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package draws problem data only.  It holds none of the solver's
arithmetic: it samples A, Q and a planted primal-dual optimum (x*, y*, z*)
and then sets b = A x* and c = A^T y* + z* - Q x*, which is the definition of
a planted instance of the separable QP (P)/(D) of the paper's introduction.
The SVM and portfolio generators write those problems in the form (P~)
with free and box-constrained variables (a change of variables and added
slacks, no solver steps).  Both the HIP path and the CPU oracle receive
exactly these arrays.
"""

from .planted import CONFIGS, Instance, make_instance, portfolio_instance, random_feasible_instance, svm_instance

__all__ = ["CONFIGS", "Instance", "make_instance", "portfolio_instance", "random_feasible_instance", "svm_instance"]
