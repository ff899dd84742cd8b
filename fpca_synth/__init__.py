"""Seeded synthetic inputs for the multi-dimensional FPCA hot path.

This module draws data from the Karhunen-Loeve model of the paper (Section 2,
eqs. 2.1-2.2): X(t) = mu(t) + sum_l A_l phi_l(t), observed with noise at points
t_ij. It holds none of the estimation arithmetic (no binning, smoothing or
eigensolving): both the HIP library's tests and the CPU oracle consume what it
produces, and nothing here depends on either of them.
"""
from .generators import (  # noqa: F401
    Dataset,
    make_config,
    make_c1,
    make_c2,
    make_c3,
    make_c4,
    make_surrogate_dataset,
    make_sim2,
    sim2_eigfun,
    irregular_kl,
    fourier_1d,
    grid_nodes,
    grid_points,
    matern15,
    C2_INDEX,
    C4_INDEX,
    fold_assignment,
    disk_time_mask,
)
