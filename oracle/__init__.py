"""FP64 CPU oracle (test infrastructure only; see excursion_set.py, two_population.py,
likelihood.py and sampler.py)."""
from .excursion_set import *  # noqa: F401,F403
from .excursion_set import Physics, Evaluation  # noqa: F401
from . import likelihood  # noqa: F401
from . import two_population  # noqa: F401
from . import sampler  # noqa: F401
