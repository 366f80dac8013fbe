"""CPU FP64 oracle for LOR assembly -- test infrastructure only (see lor_oracle)."""
from .lor_oracle import *  # noqa: F401,F403
