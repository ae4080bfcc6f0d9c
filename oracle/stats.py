"""Batch statistics (oracle; test infrastructure only).

Per-step metrics of the paper's benchmark are throughput only (Sec. VI); the
statistics here are this framework's health summary of a batch: vehicles
with a non-finite state, mean position error of position-mode vehicles, mean
body-rate norm, saturated rotor commands and resets.  Non-finite vehicles
are left out of the means.
"""
import torch


def final_state_stats(state, mode, target):
    finite = torch.isfinite(state).all(-1)
    pos = (torch.as_tensor(mode) == 0) & finite
    err = torch.linalg.vector_norm(state[:, 0:3] - target[:, 0:3], dim=-1)
    wn = torch.linalg.vector_norm(state[:, 10:13], dim=-1)
    return {
        "n_nonfinite": int((~finite).sum()),
        "n_position": int(pos.sum()),
        "pos_err_sum": float(err[pos].sum()),
        "n_finite": int(finite.sum()),
        "omega_sum": float(wn[finite].sum()),
    }
