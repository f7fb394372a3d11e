"""Independent reader of the GPU word layout, used to check the host builder on the CPU.

It walks the buffer as the layout is documented (hvf_build.cpp header) and lists every
occupied voxel, so a test can compare the result with the builder's input. It shares no
code with the library.
"""
import numpy as np


def _depths(info):
    """Per traversal depth: (level, kind, j, L, cs, w) from the level list."""
    kinds = info["kinds"]
    exps = info["level_exp"]
    n = len(kinds)
    sub = [0] * (n + 1)
    for k in range(n - 1, 0, -1):
        sub[k] = sub[k + 1] + exps[k][0]
    out = []
    for k in range(n):
        if kinds[k] == "R" and k < n - 1:
            out.append((k, "R", 0, 1, sub[k + 1], exps[k]))
        elif kinds[k] == "R":
            out.append((k, "B", 0, 1, 0, exps[k]))  # last Raw level: a brick of 64-bit block masks
        else:
            L = exps[k][0]
            for j in range(L):
                out.append((k, kinds[k], j, L, sub[k + 1] + (L - 1 - j), (1, 1, 1)))
    return out, n


def decode(info, words):
    """Return the sorted list of occupied voxels (x, y, z)."""
    W = [int(v) for v in words] if len(words) < 200000 else words
    D, nlev = _depths(info)
    out = []
    root = int(W[0])
    if root == 0:
        return out

    def enter(d, ptr):
        k, kind, j, L, cs, w = D[d]
        if kind in ("R", "B"):
            return ptr, 0xFF
        if kind == "S":
            return int(W[ptr]), int(W[ptr + 1]) & 0xFF
        return ptr + 1, int(W[ptr]) & 0xFF

    def walk(d, ptr, corner):
        k, kind, j, L, cs, w = D[d]
        last_level = (k == nlev - 1)
        base, valid = enter(d, ptr)
        if kind == "B":
            # blocks of side 2^b (b = min(2, smallest exponent)), blocks x-fastest, one
            # 64-bit mask per block with bits x-fastest inside the block
            b = min(2, min(w))
            bx, by, bz = w[0] - b, w[1] - b, w[2] - b
            for blk in range(1 << (bx + by + bz)):
                m = int(W[ptr + 2 * blk]) | (int(W[ptr + 2 * blk + 1]) << 32)
                ox, oy, oz = blk & ((1 << bx) - 1), (blk >> bx) & ((1 << by) - 1), blk >> (bx + by)
                for bit in range(64):
                    if (m >> bit) & 1:
                        cx, cy, cz = bit & ((1 << b) - 1), (bit >> b) & ((1 << b) - 1), bit >> (2 * b)
                        assert cz < (1 << b), "bit beyond the block"
                        out.append((corner[0] + (ox << b) + cx, corner[1] + (oy << b) + cy, corner[2] + (oz << b) + cz))
            return
        if kind == "R":
            wx, wy, wz = w
            ncell = 1 << (wx + wy + wz)
            for idx in range(ncell):
                p = int(W[base + idx])
                if p:
                    cx, cy, cz = idx & ((1 << wx) - 1), (idx >> wx) & ((1 << wy) - 1), idx >> (wx + wy)
                    walk(d + 1, p, (corner[0] + (cx << cs), corner[1] + (cy << cs), corner[2] + (cz << cs)))
            return
        deepest = (j == L - 1)
        for o in range(8):
            if not (valid >> o) & 1:
                continue
            c = (corner[0] + ((o & 1) << cs), corner[1] + (((o >> 1) & 1) << cs), corner[2] + (((o >> 2) & 1) << cs))
            rank = bin(valid & ((1 << o) - 1)).count("1")
            if deepest and last_level:
                out.append(c)
            elif kind == "S" and not deepest:
                walk(d + 1, base + 2 * rank, c)
            elif kind == "G" and not deepest:
                # descriptor: (child pointer, copy of the child's mask word)
                child = int(W[base + 2 * rank])
                assert int(W[base + 2 * rank + 1]) == int(W[child]), "descriptor mask differs from the child's"
                walk(d + 1, child, c)
            else:
                walk(d + 1, int(W[base + rank]), c)

    walk(0, root, (0, 0, 0))
    out.sort(key=lambda v: (v[2], v[1], v[0]))
    return out


def decode_codes(info, words, morton_encode):
    v = decode(info, words)
    if not v:
        return np.zeros(0, np.uint64)
    return np.sort(morton_encode(np.array(v, dtype=np.int32)))
