"""Seeded synthetic inputs shared by the oracle and the GPU engine.

Holds the colour-code geometry and the op-list builder (what the circuit is),
nothing of how it is simulated."""
from .colorcode import ColorCode, build_color_code, gf2_rank  # noqa: F401
from .circuit import (Circuit, build_circuit, custom_circuit, random_program,  # noqa: F401
                      default_layout, snake_layout, edge_colouring,
                      n_leaves_for, ops_per_shot, uniform_params, CHANNELS,
                      OP_INIT, OP_CNOT, OP_SRX, OP_AD, OP_PAULI, OP_MEAS, OP_NAMES,
                      C_OP, C_Q0, C_Q1, C_ARG, C_LOC, C_DRAW, C_REC, C_PREV, C_TICK, N_COLS)
from .layout import exact_bond_dim, optimized_layout, clustered_layout, similarity_matrix  # noqa: F401,E402
