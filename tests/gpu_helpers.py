"""Helpers of the GPU tests (written independently of the library)."""
import numpy as np


def unpack_spins(packed: np.ndarray, n: int) -> np.ndarray:
    """Packed uint64 rows (bit i of word i//64 set <=> s_i = -1) -> int8 +1/-1 rows."""
    packed = np.ascontiguousarray(packed).view(np.uint64)
    out = np.empty((packed.shape[0], n), np.int8)
    for i in range(n):
        bit = (packed[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)
        out[:, i] = np.where(bit == 1, -1, 1)
    return out


def pack_spins(spins: np.ndarray) -> np.ndarray:
    """int8 +1/-1 rows -> packed uint64 rows, returned as int64 (torch has no uint64)."""
    count, n = spins.shape
    words = (n + 63) // 64
    out = np.zeros((count, words), np.uint64)
    for i in range(n):
        out[:, i // 64] |= (spins[:, i] < 0).astype(np.uint64) << np.uint64(i % 64)
    return out.view(np.int64)


def rel_inf_error(x_gpu: np.ndarray, x_ref: np.ndarray) -> np.ndarray:
    """Per (row, step): max_i |x_gpu - x_ref| / max_i |x_ref|."""
    num = np.abs(x_gpu.astype(np.float64) - x_ref).max(axis=-1)
    den = np.abs(x_ref).max(axis=-1)
    return num / np.maximum(den, 1e-30)
