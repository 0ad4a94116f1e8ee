"""Seeded synthetic inputs shared by the oracle tests and the GPU library tests."""
from .problems import (CONFIGS, batch_sizes, config_problem, family_member, interior_iterate,
                       kkt_state, make_problem)

__all__ = ["CONFIGS", "batch_sizes", "config_problem", "family_member", "interior_iterate",
           "kkt_state", "make_problem"]
