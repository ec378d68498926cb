"""Test-side conversion of a workload dict into the oracle's Model."""

import numpy as np

from oracle.qhfpe_oracle import Model


def oracle_model(d: dict) -> Model:
    return Model(
        n_states=d["n_states"], nq=d["nq"], np_=d["np"],
        q_min=d["q_min"], q_max=d["q_max"], p_min=d["p_min"], p_max=d["p_max"],
        depth=d["depth"], zeta=d["zeta"], gamma=d["gamma"], beta=d["beta"], dt=d["dt"],
        poly=np.array(d["poly"], dtype=np.float64), mu=np.array(d["mu"], dtype=np.float64),
        mass=d.get("mass", 1.0), hbar=d.get("hbar", 1.0),
        low_temp_correction=d.get("low_temp_correction", True),
    )


def single_state(poly1d, **kw):
    """A one-state workload dict with potential coefficients poly1d."""
    base = dict(n_states=1, nq=64, np=64, q_min=-8.0, q_max=8.0, p_min=-8.0, p_max=8.0,
                depth=0, zeta=0.0, gamma=1.0, beta=1.0, dt=0.005,
                poly=[[list(poly1d) + [0.0] * (5 - len(poly1d))]], mu=[[0.0]],
                mass=1.0, hbar=1.0, low_temp_correction=True)
    base.update(kw)
    return base


def top_window(d: dict, k: int) -> dict:
    """The model on the top k q columns of d's grid: same spacing, same upper
    end, q_min moved up by nq - k columns."""
    dq = (d["q_max"] - d["q_min"]) / d["nq"]
    out = dict(d)
    out.update(nq=k, q_min=d["q_min"] + (d["nq"] - k) * dq)
    return out
