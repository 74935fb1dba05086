"""The oracle's default options follow the paper's option set (Sec. 3, the
option list of the results), except the overrides the workload names."""
import os

from oracle.params import Params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_option_set.txt")


def read_option_set():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            parts = line.split()
            out[parts[0]] = float(parts[1])
    return out


def test_oracle_defaults_follow_the_paper_option_set():
    p = Params()
    for k, v in read_option_set().items():
        assert float(getattr(p, k)) == v, k
