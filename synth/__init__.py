from .workloads import *  # noqa: F401,F403
from .workloads import SEED, ALPHA, BETA, WORKLOADS, Problem, make_problem, config, batch_shapes, batch_utterance  # noqa: F401
