"""Shared helpers of the tests: lockstep GPU/oracle rollouts and error metrics."""
import numpy as np


def oracle_tools(tools):
    """Tool dicts for the oracle: every tool keeps its index (history slot)."""
    return [dict(t, contact=int(bool(t.get("contact"))), cutting=int(bool(t.get("cutting")))) for t in tools]


def oracle_substep(o, tools):
    blades = [t["blade"] for t in tools if t.get("labels")]
    if blades:
        o.assign_labels(blades)
    st, w = o.step(oracle_tools(tools))
    return st, w


def field_err(a, b):
    """max_p ||a_p - b_p||_inf / max_p ||b_p||_inf (scene-relative)."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def disp_err(x_gpu, x_orc, X):
    """max_p ||x_gpu - x_orc|| / max_p ||x_orc - X|| (displacement-relative)."""
    num = np.linalg.norm(np.asarray(x_gpu, np.float64) - x_orc, axis=1).max()
    den = np.linalg.norm(x_orc - np.asarray(X, np.float64), axis=1).max()
    return num / den


def gpu_x(state, X):
    return np.asarray(X, np.float64) + state["u"].astype(np.float64)
