"""FP64 CPU oracle for PID (test infrastructure only; see ``pid_oracle``)."""
from .pid_oracle import *  # noqa: F401,F403
from .pid_oracle import __all__  # noqa: F401
