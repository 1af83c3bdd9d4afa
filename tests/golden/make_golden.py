"""Writes the closed-form fixtures under tests/golden/.

Only formulas stated in the paper are evaluated here:
  * Eq. (6): the Pauli-twirled ZZ crosstalk channel flips with probability
    sin^2(theta).  For one exp(-i theta Z Z) on |++> followed by an X-basis
    measurement of the first qubit, the flip outcome has exactly that
    probability (the coherent channel and its twirl agree on this single
    event).
  * Eqs. (2)-(3): the depolarising channels pick each non-identity Pauli with
    probability p/3 (one qubit) and p/15 (two qubits).
  * Table I: the error-rate ratios per location kind (single-qubit gate
    0.1 p, two-qubit gate p, reset 2 p, measurement 5 p).
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    thetas = [1e-3, 0.02, 0.05, 0.1, 0.3, math.pi / 4, 1.0]
    eq6 = {"citation": "Eq. (6), Pauli twirling approximation of Eq. (4): flip probability sin^2(theta)",
           "cases": [{"theta": t, "p_flip": math.sin(t) ** 2} for t in thetas]}
    with open(os.path.join(HERE, "eq6_single_rotation.json"), "w") as f:
        json.dump(eq6, f, indent=1)
    dep = {"citation": "Eqs. (2)-(3): p/3 per single-qubit Pauli, p/15 per two-qubit Pauli pair",
           "one_qubit": {"k": 3, "each": "p/3"}, "two_qubit": {"k": 15, "each": "p/15"},
           "table_I": {"citation": "Table I: error rates relative to the parameter p",
                       "single_qubit_gate": 0.1, "two_qubit_gate": 1.0, "reset": 2.0, "measurement": 5.0}}
    with open(os.path.join(HERE, "eq2_eq3_depolarizing.json"), "w") as f:
        json.dump(dep, f, indent=1)


if __name__ == "__main__":
    main()
