"""CPU oracle -- test infrastructure only (see ``ref.py``)."""
from .ref import *  # noqa: F401,F403
from .ref import num_threads, set_num_threads  # noqa: F401
