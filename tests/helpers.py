"""Shared test helpers: layout conversion between the library's [band][i][G]
(G in library order, rows padded to ld) and the oracle's [band][G*Nb + i]."""
import numpy as np


def gperm(lib_m: np.ndarray, oracle_m: np.ndarray) -> np.ndarray:
    """perm[g_lib] = index of the same (m1, m2) in the oracle's G list."""
    pos = {(int(a), int(b)): n for n, (a, b) in enumerate(oracle_m)}
    return np.array([pos[(int(a), int(b))] for a, b in lib_m])


def lib_to_oracle(x_lib: np.ndarray, ng: int, perm: np.ndarray) -> np.ndarray:
    """x_lib [nb_vec][nb][ld] -> oracle vectors [nb_vec][ng*nb]."""
    nv, nb, _ = x_lib.shape
    out = np.zeros((nv, ng, nb), dtype=np.complex128)
    out[:, perm, :] = np.transpose(x_lib[:, :, :ng], (0, 2, 1))
    return out.reshape(nv, ng * nb)


def oracle_to_lib(x: np.ndarray, nb: int, ng: int, ld: int, perm: np.ndarray) -> np.ndarray:
    nv = x.shape[0]
    xr = x.reshape(nv, ng, nb)
    out = np.zeros((nv, nb, ld), dtype=np.complex128)
    out[:, :, :ng] = np.transpose(xr[:, perm, :], (0, 2, 1))
    return out


def random_lib_block(seed: int, nv: int, nb: int, ng: int, ld: int) -> np.ndarray:
    from paper_1406_4960_amd import workloads
    x = np.zeros((nv, nb, ld), dtype=np.complex128)
    x[:, :, :ng] = workloads.random_block(seed, nv, nb, ng)
    return x


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
