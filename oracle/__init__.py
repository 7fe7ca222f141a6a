"""CPU oracle of the double FFT filter -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never calls it.
"""
from .oracle import (EXP, GAUSS, SHARP, HYBRID, mask, theta_cutoff, phi_cutoff, sin_theta,
                     theta_pass, phi_pass, forward, adjoint, lib_path, set_detector,
                     shock_detected, decisions, set_threads)

__all__ = ["EXP", "GAUSS", "SHARP", "HYBRID", "mask", "theta_cutoff", "phi_cutoff", "sin_theta",
           "theta_pass", "phi_pass", "forward", "adjoint", "lib_path", "set_detector",
           "shock_detected", "decisions", "set_threads"]
