"""FP64 CPU oracle for the FOT hot path (test infrastructure only; see fot_oracle)."""
from .fot_oracle import *  # noqa: F401,F403
from .fot_oracle import __all__  # noqa: F401
from . import beam  # noqa: F401,E402  (output beam and Gerchberg-Saxton polishing)
from . import cfot  # noqa: F401,E402  (FFT-convolution variant of the iteration, Eq. 11)
