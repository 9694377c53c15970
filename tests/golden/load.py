"""Reader of the hand-derived text fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _row(fields):
    return [complex(float(a), float(b)) for a, b in (f.split(",") for f in fields)]


def theta_identity_rows() -> dict:
    """Cases of theta_identity_rows.txt: {name: dict(phi, psi, theta, idx)}."""
    cases, cur = {}, None
    for line in open(os.path.join(HERE, "theta_identity_rows.txt")):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, *fields = line.split()
        if key == "case":
            cur = cases.setdefault(fields[0], {"phi": [], "psi": [], "theta": []})
        else:
            cur[key].append(_row(fields))
    out = {}
    for name, c in cases.items():
        phi = np.array(c["phi"], dtype=np.complex128)
        psi = np.array(c["psi"], dtype=np.complex128) if c["psi"] else phi
        out[name] = dict(phi=phi, psi=psi, theta=np.array(c["theta"], dtype=np.complex128),
                         idx=np.array([0, 1], dtype=np.int32))
    return out
