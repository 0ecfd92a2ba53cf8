"""Reader for tests/golden/paper_values.txt (values quoted from the paper)."""
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def paper_values():
    vals = {}
    with open(_PATH) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            vals[k] = float(v)
    return vals
