"""Small binary linear codes built for tests (input construction only)."""
import numpy as np

import synth


def small_code(n, k, even, seed):
    """A systematic [n, k] code with a random parity part, no bit that is 0 in every codeword, and
    rows of even weight (an even code) when `even`."""
    rng = np.random.default_rng(seed)
    while True:
        P = rng.integers(0, 2, size=(k, n - k)).astype(np.uint8)
        if even:
            P[:, -1] = (1 + P[:, :-1].sum(1)) % 2
        elif np.all((1 + P.sum(1)) % 2 == 0):
            P[0, -1] ^= 1
        if np.all(P.any(0)):
            break
    G = np.concatenate([np.eye(k, dtype=np.uint8), P], axis=1)
    return synth.code_from_generator(f"[{n},{k}]{'e' if even else ''}", G, list(range(k)))
