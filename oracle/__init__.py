"""FP64 CPU oracle of the fused lattice-Boltzmann LES canopy step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP library (see ``lbm_ref.c`` for the method and readings).
"""
