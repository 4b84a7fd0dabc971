"""Python int <-> little-endian uint32 limb arrays (marshalling only)."""
from __future__ import annotations

from typing import Iterable, Sequence

import numpy as np


def limbs_needed(x: int) -> int:
    return max(1, (x.bit_length() + 31) // 32)


def to_limbs(values: Sequence[int] | int, nlimbs: int) -> np.ndarray:
    """Pack non-negative ints into a ``[count][nlimbs]`` uint32 array (LE limbs).

    A scalar int gives a 1-D ``[nlimbs]`` array.
    """
    scalar = isinstance(values, (int, np.integer))
    vals = [int(values)] if scalar else [int(v) for v in values]
    nbytes = 4 * nlimbs
    buf = bytearray(len(vals) * nbytes)
    for i, v in enumerate(vals):
        if v < 0 or v.bit_length() > 32 * nlimbs:
            raise ValueError(f"value does not fit in {nlimbs} limbs")
        buf[i * nbytes:(i + 1) * nbytes] = v.to_bytes(nbytes, "little")
    arr = np.frombuffer(bytes(buf), dtype="<u4").reshape(len(vals), nlimbs)
    arr = arr.astype(np.uint32, copy=True)
    return arr[0] if scalar else arr


def from_limbs(arr: np.ndarray) -> int:
    """One little-endian limb vector -> int."""
    a = np.ascontiguousarray(arr, dtype="<u4")
    return int.from_bytes(a.tobytes(), "little")


def ints_from_limbs(arr: np.ndarray) -> list[int]:
    """``[count][nlimbs]`` -> list of ints."""
    a = np.ascontiguousarray(arr, dtype="<u4")
    if a.ndim == 1:
        return [from_limbs(a)]
    nb = 4 * a.shape[1]
    raw = a.tobytes()
    return [int.from_bytes(raw[i * nb:(i + 1) * nb], "little") for i in range(a.shape[0])]


def u64_to_ints(arr: Iterable) -> list[int]:
    return [int(v) for v in np.asarray(arr, dtype=np.uint64)]
