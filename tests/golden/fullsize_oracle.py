"""Shared writer and reader of the full-size oracle fixtures.

A fixture holds the FP64 oracle's solve of one workload: scalars of the last
check, the relative error at every recorded check, the singular values of the
SVD init and a seeded sample of rows of the final U and V.  Both writers
(make_image_oracle.py, make_ratings_oracle.py) call only the oracle and the
seeded input generators.
"""

import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

SCALARS = ("f", "relerr", "re_paper", "kkt", "relerr_svd", "iters", "ext_iters_done", "converged",
           "rot_steps", "neg_mass_before", "neg_mass_after", "step_u", "step_v")


def sample_rows(count, total, seed):
    """The rows whose values a fixture stores (sorted, without repeats)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=min(count, total), replace=False))


def write(name, header, rep, U, V, rows_u, rows_v, seconds):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        f.write(f"# written in {seconds:.0f} s\n")
        for key in SCALARS:
            v = rep[key]
            f.write(f"{key} {float(v)!r}\n")
        f.write("sigma " + " ".join(repr(float(s)) for s in rep["sigma"]) + "\n")
        for c in rep["checks"]:
            f.write(f"check {int(c['k'])} {float(c['relerr'])!r} {float(c['kkt'])!r}\n")
        for i in rows_u:
            f.write(f"U {int(i)} " + " ".join(repr(float(x)) for x in U[i]) + "\n")
        for j in rows_v:
            f.write(f"V {int(j)} " + " ".join(repr(float(x)) for x in V[j]) + "\n")
    return path


def read(name):
    """dict with the scalars, 'sigma', 'checks' (k, relerr, kkt rows) and the
    sampled rows 'U', 'V' as (indices, values)."""
    out = {"checks": [], "U": ([], []), "V": ([], [])}
    for line in open(os.path.join(HERE, name)):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        if tok[0] == "sigma":
            out["sigma"] = np.array([float(t) for t in tok[1:]])
        elif tok[0] == "check":
            out["checks"].append((int(tok[1]), float(tok[2]), float(tok[3])))
        elif tok[0] in ("U", "V"):
            out[tok[0]][0].append(int(tok[1]))
            out[tok[0]][1].append([float(t) for t in tok[2:]])
        else:
            out[tok[0]] = float(tok[1])
    for key in ("U", "V"):
        out[key] = (np.array(out[key][0], dtype=np.int64), np.array(out[key][1]))
    out["checks"] = np.array(out["checks"])
    return out


def timed(fn):
    t0 = time.perf_counter()
    res = fn()
    return res, time.perf_counter() - t0
