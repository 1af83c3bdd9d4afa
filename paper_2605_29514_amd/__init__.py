"""MI355X-native hot path of the hybrid stabilizer-tensor-network simulator
for surface codes under coherent crosstalk (Harper, Nakhl, Sevior, Usman).

Submodules:
  workload  seeded synthetic circuits and uniforms (inputs only)
  stn       ctypes binding of the C-ABI library libstn.so (HIP kernels)
"""
