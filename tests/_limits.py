"""Largest domains the library accepts: each state buffer (nine population
planes, plus the FP32 density plane of the FP16 per-node form) must stay
below 4 GiB, since the kernels address it with 32-bit byte offsets.  Plane
layout: rows of pitch = nx rounded up to 64 elements, planes staggered by
256 elements."""

BYTES = {"f64": 8, "f32": 4, "f32_arith32": 4, "f32dev": 4, "f16dev": 2, "f16node": 2}
LIMIT = (1 << 32) - 256


def buffer_bytes(storage: str, nx: int, ny: int) -> int:
    pitch = (nx + 63) // 64 * 64
    plane = pitch * ny + 256
    extra = 4 * plane if storage == "f16node" else 0
    return 9 * plane * BYTES[storage] + extra


def max_rows(storage: str, nx: int) -> int:
    """The largest ny whose state buffer fits (nx * ny must also stay below
    2^30 nodes)."""
    ny = 0
    lo, hi = 1, (1 << 30) // nx
    while lo <= hi:
        mid = (lo + hi) // 2
        if buffer_bytes(storage, nx, mid) < LIMIT:
            ny, lo = mid, mid + 1
        else:
            hi = mid - 1
    return ny
