"""Seeded synthetic inputs shared by the oracle tests and the GPU drivers."""
from .splitmix import draw, mix64, stream_seed, unit, randint  # noqa: F401
from .generators import (  # noqa: F401
    Diagram, batch_diagram, batch_params, bernoulli_matrix, bernoulli_rows,
    make_diagram, pack_rows, pauli_strings, poisson_arrivals, single_diagram,
    unpack_rows, words_for,
)
