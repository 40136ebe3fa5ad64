"""CPU oracle for the lattice-sum method (test infrastructure only; see lattice_oracle)."""
from .lattice_oracle import *  # noqa: F401,F403
