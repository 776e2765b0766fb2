"""Reader for the text fixtures in tests/golden/ (values printed in the paper).

Entries are arithmetic expressions over numbers, ``pi`` and ``sqrt``; they are
evaluated with no builtins available."""
import math
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_ENV = {"__builtins__": {}, "sqrt": math.sqrt, "pi": math.pi}


def _value(expr):
    return float(eval(expr, _ENV))  # noqa: S307 -- restricted arithmetic only


def load_sections(name):
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                out[cur] = []
                continue
            out.setdefault(cur, []).append([_value(x) for x in line.split()])
    return out
