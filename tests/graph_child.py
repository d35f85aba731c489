"""Child process of test_graph_replays_match_eager: the same preconditioner
applications and matvecs with HIP graphs off (H2SP_GRAPHS=0, set by the
parent), saved for a bitwise comparison."""
import sys

import numpy as np

sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import paper_1705_04601_amd as P  # noqa: E402
from graph_cases import run_sequence  # noqa: E402

np.save(sys.argv[2], run_sequence(P))
