"""Seeded initial weights of the learned level-of-detail network.

The random numbers of training start here, as an input: He-uniform weights
(bound sqrt(6 / fan_in)) and zero biases, in the parameter order W1[32][8],
b1[32], W2[32][32], b2[32], w3[32], b3, rounded to FP32.
"""
import numpy as np

N_IN, N_H = 8, 32
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def mlp_init(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, N_H * N_IN) * np.sqrt(6.0 / N_IN), np.zeros(N_H),
             rng.uniform(-1, 1, N_H * N_H) * np.sqrt(6.0 / N_H), np.zeros(N_H),
             rng.uniform(-1, 1, N_H) * np.sqrt(6.0 / N_H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
