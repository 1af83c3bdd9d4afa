"""Plain FP64 CPU oracle for the hybrid stabilizer-tensor-network (STN) step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything here: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; the only thing both sides read is the seeded workload generator.

Modules:
  tableau      Pauli strings and the inverse Clifford tableau (Sec. IV.A, Eq. 7)
  mps          matrix-product state, two-term operator application, QR/SVD
               compression and truncation (Sec. IV.B, Eq. 8)
  stn          one shot of the STN simulation over a circuit (Sec. IV.A)
  statevector  brute-force physical simulation (pins stn without truncation)
  chp          Aaronson-Gottesman stabilizer simulation (pins theta = 0 runs)
  grad         frozen-projector log-probability gradient
"""
