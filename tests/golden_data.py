"""Loader for the text fixtures under tests/golden/ (each row cites its source)."""
import os

_HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load_soils():
    out = {}
    with open(os.path.join(_HERE, "soils.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            name, *vals = line.split()
            out[name] = tuple(float(v) for v in vals)
    return out


SOILS = _load_soils()
