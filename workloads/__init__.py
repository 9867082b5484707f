"""Seeded synthetic inputs shared by the oracle tests and the GPU drivers."""
from .splitmix import draw, mix64, stream_seed, unit, randint  # noqa: F401
from .generators import (  # noqa: F401
    Diagram, batch_diagram, batch_params, bernoulli_matrix, bernoulli_rows,
    make_diagram, network_init, pack_rows, parity_problem, ParityProblem, surface_dem, DetectorModel, param_rows, pauli_strings, poisson_arrivals, serve_diagram,
    serve_params, single_diagram, unpack_rows, words_for,
)
