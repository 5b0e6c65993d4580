"""libasp for MI355X (gfx950): the data-parallel search of the conflict-driven
ASP solver of Dovier, Formisano and Vella, "GPU-based parallelism for
ASP-solving", as hand-written HIP behind a C ABI (include/asp.h).

``binding`` marshals arguments to the library; ``build`` compiles it.
"""
from .binding import (Batch, Program, AspError, limits, options, lib,  # noqa: F401
                      scorer_weights, SAT, UNSAT, UNKNOWN, FIXPOINT, CONFLICT, RUNNING,
                      DECISION_OCC, DECISION_SCORE, DECISION_JW,
                      DECISION_ACTIVITY, LEARN_FWD, LEARN_RES)
