"""Seeded synthetic inputs shared by the oracle tests and the GPU library tests."""
from .problems import (CONFIGS, IPM_N192, LARGE_N16384, OPF_N4096, batch_sizes, config_problem, family_member, interior_iterate,
                       kkt_state, make_problem, nlp_terms, sparse_blocks)

__all__ = ["CONFIGS", "IPM_N192", "LARGE_N16384", "OPF_N4096", "batch_sizes", "config_problem", "family_member", "interior_iterate",
           "kkt_state", "make_problem", "nlp_terms", "sparse_blocks"]
