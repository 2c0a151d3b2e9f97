"""Seeded synthetic cryo-ET inputs shared by the GPU path's tests and the oracle.

This module only draws inputs: blob templates, Haar-random rotations, the
missing-wedge mask, noise and starting rotations.  It holds none of the
ball-harmonic arithmetic (no basis, expansion, Wigner matrix or score).

Recipe (stand-in for the paper's SHREC 2020 tomograms, which are not
available): a template is a sum of isotropic Gaussian blobs
A_j exp(-|x - c_j|^2 / (2 sigma^2)) with sigma = 0.1 in the [-1, 1]^3 box
(5 % of the box side), amplitudes A_j ~ U[0.5, 1] and centres uniform in the
ball of radius 0.8.  A particle is the template rotated by a Haar-random
g* (analytically: centres c_j -> g* c_j, so f(x) = t(g*^{-1} x)), then
restricted to a +/- tilt missing wedge about the y axis in Fourier space
(beam along z: keep |k_z| <= tan(tilt) |k_x|), then white Gaussian noise of
variance var(wedged volume) / SNR is added.  Volumes are cell-centred samples
x_i = (i - (N-1)/2) * 2/N, ``vol[i, j, k]`` at (x_i, y_j, z_k), stored FP32.
"""

from .volumes import (  # noqa: F401
    seed_rng, haar_quaternions, quat_to_matrix, matrix_to_euler_zyz,
    euler_zyz_to_matrix, blob_template, render_blobs, wedge_mask,
    apply_wedge, add_noise, make_particles, random_starts, Workload,
    CONFIG1, CONFIG2,
)
