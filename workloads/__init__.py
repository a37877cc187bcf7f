"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
golden-value script.

This module only draws random numbers and plants known answers. It holds none
of the method's arithmetic (no distances, no normalisation, no screening), so
the GPU path and the CPU oracle can both consume its output without sharing
any code that computes a result.
"""
from .synth import (  # noqa: F401
    MASTER_SEED,
    config_rng,
    gaussian_points,
    planted_gaussian_points,
    random_walk,
    plant_motif,
    mixture_points,
    snp_matrix,
    plant_snp_pairs,
    batch_series,
    cfg_points_small,
    cfg_motif,
    cfg_walk,
    cfg_strings,
    cfg_two_locus,
    random_strings,
    plant_string_pair,
    noise_genotypes,
    inject_two_locus_pair,
    cfg_mixture,
    cfg_batch,
    cfg_snp,
    valid_pairs_points,
    valid_pairs_motif,
)
