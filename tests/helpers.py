"""Shared helpers of the test-suite: build the oracle and the GPU library from one
parameter set, run both, and measure field errors."""

import numpy as np

from oracle import lbm as olbm

MOMENT_NAMES = ("phi", "cA", "cB", "muA", "muB", "p", "ux", "uy", "uz")


def oracle_params(p):
    return olbm.Params(**p)


def gpu_config(p, precision, **kw):
    from paper_2409_03401_amd.lbm import LBMConfig
    return LBMConfig(**p, precision=precision, **kw)


def oracle_run(p, phi0, muA0, muB0, steps):
    prm = oracle_params(p)
    st = olbm.init(phi0, muA0, muB0, prm)
    st = olbm.run(st, prm, steps)
    return prm, st


def oracle_moments(prm, st):
    m = olbm.moments(st, prm)
    return {k: np.asarray(m[k]) for k in MOMENT_NAMES}


def oracle_populations(prm, st):
    parts = []
    if st.f is not None:
        parts.append(st.f)
    parts += [st.g, st.hA, st.hB]
    return np.concatenate(parts, axis=0)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return num / den if den > 0 else num


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))))


def field_errors(gpu, ora, names=MOMENT_NAMES):
    return {k: (rel_l2(gpu[k], ora[k]), max_abs(gpu[k], ora[k])) for k in names}
