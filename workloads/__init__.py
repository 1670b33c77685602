"""Seeded synthetic inputs for the GKR prover: circuits and their input data.

This package holds the input generators only: SplitMix64 draws of the data
vectors and the wiring of the benchmark circuits (F2, MatMult, pattern
matching, and F0 with the F0-based single-output PM and MatMult checks).
It performs none of the protocol's arithmetic, so both the CPU oracle's
tests and the GPU path may take their inputs from it.
"""
from .prng import splitmix64, uniform_bits, PURPOSE
from .circuits import (Circuit, f2_circuit, matmult_circuit, pm_circuit, f0_circuit,
                       pm_f0_circuit, matmult_check_circuit)
from .configs import (f2_inputs, matmult_inputs, pm_inputs, f2sc_vector, f0_inputs,
                      matmult_check_inputs, c1_f2, c2_f2, c2_f2sc, c3_matmult, batch_mix,
                      f1_f0, f1_pm_f0, f1_matmult_check, P)

__all__ = ["splitmix64", "uniform_bits", "PURPOSE", "Circuit", "f2_circuit",
           "matmult_circuit", "pm_circuit", "f2_inputs", "matmult_inputs",
           "pm_inputs", "f2sc_vector", "c1_f2", "c2_f2", "c2_f2sc",
           "c3_matmult", "batch_mix", "P", "f0_circuit", "pm_f0_circuit",
           "matmult_check_circuit", "f0_inputs", "matmult_check_inputs", "f1_f0",
           "f1_pm_f0", "f1_matmult_check"]
