"""The paper's matrix-vector (MV) cost model (oracle; test infrastructure).

Paper, Sec. 5 ("Results"), paragraph on MV operations:
  * CG with a Chebyshev polynomial of degree d: 2d MV for the polynomial plus
    2 for M^dagger M itself, i.e. 2(d+1) per iteration;
  * CG with the strong-coupling preconditioner: about 3 MV per iteration;
  * BiCGStab with the weak-coupling preconditioner of order d:
    2(d+1)(1+2 beta) MV per iteration, beta = 1 in the tables.
"""


def mv_per_iteration(method: str, degree: int = 0, beta: float = 1.0) -> float:
    if method == "cheb":
        return 2 * (degree + 1)
    if method == "sca":
        return 3
    if method == "wce":
        return 2 * (degree + 1) * (1 + 2 * beta)
    if method == "none":
        return 2
    raise ValueError(method)


def mv_count(method: str, iterations: int, degree: int = 0, beta: float = 1.0) -> float:
    return iterations * mv_per_iteration(method, degree, beta)
