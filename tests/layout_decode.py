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
        if kinds[k] in "RD" and k < n - 1:
            # DF pointer grid: one word per cell, top bit set = empty (low bits: distance)
            out.append((k, kinds[k], 0, 1, sub[k + 1], exps[k]))
        elif kinds[k] in "RD":
            # last Raw level: a brick of 64-bit block masks; a last DF level with more than
            # one block stores 4 words per block (mask lo, mask hi, block distance, 0)
            b = min(2, min(exps[k]))
            many = sum(e - b for e in exps[k]) > 0
            out.append((k, "E" if kinds[k] == "D" and many else "B", 0, 1, 0, exps[k]))
        else:
            L = exps[k][0]
            for j in range(L):
                out.append((k, kinds[k], j, L, sub[k + 1] + (L - 1 - j), (1, 1, 1)))
    return out, n


def decode(info, words):
    """Return the sorted list of occupied voxels (x, y, z). With per-depth regions
    (info["depth_buffers"]) every pointer is relative to the start of the region of the
    depth it points into: the next depth's, or for an SVO node's pointer array its own."""
    W = [int(v) for v in words] if len(words) < 200000 else words
    D, nlev = _depths(info)
    out = []
    regions = info.get("depth_buffers", False)

    def rb(d):  # pointers count from 16 words before their region (0 stays the empty marker)
        return info["depth_offset"][d] - 16 if regions and d < len(D) else 0

    root = int(W[0])
    if root == 0:
        return out
    root += rb(0)

    def enter(d, ptr):
        k, kind, j, L, cs, w = D[d]
        if kind in ("R", "B", "D", "E"):
            return ptr, 0xFF
        if kind == "S":
            deepest_above = j == L - 1 and k < nlev - 1  # its pointer array lies in its own region
            return int(W[ptr]) + (rb(d) if deepest_above else rb(d + 1)), int(W[ptr + 1]) & 0xFF
        return ptr + 1, int(W[ptr]) & 0xFF

    def walk(d, ptr, corner):
        k, kind, j, L, cs, w = D[d]
        last_level = (k == nlev - 1)
        base, valid = enter(d, ptr)
        if kind in ("B", "E"):
            # blocks of side 2^b (b = min(2, smallest exponent)), blocks x-fastest, one
            # 64-bit mask per block with bits x-fastest inside the block
            b = min(2, min(w))
            bx, by, bz = w[0] - b, w[1] - b, w[2] - b
            st = 4 if kind == "E" else 2
            for blk in range(1 << (bx + by + bz)):
                m = int(W[ptr + st * blk]) | (int(W[ptr + st * blk + 1]) << 32)
                ox, oy, oz = blk & ((1 << bx) - 1), (blk >> bx) & ((1 << by) - 1), blk >> (bx + by)
                for bit in range(64):
                    if (m >> bit) & 1:
                        cx, cy, cz = bit & ((1 << b) - 1), (bit >> b) & ((1 << b) - 1), bit >> (2 * b)
                        assert cz < (1 << b), "bit beyond the block"
                        out.append((corner[0] + (ox << b) + cx, corner[1] + (oy << b) + cy, corner[2] + (oz << b) + cz))
            return
        if kind in ("R", "D"):
            wx, wy, wz = w
            ncell = 1 << (wx + wy + wz)
            for idx in range(ncell):
                p = int(W[base + idx])
                if kind == "D" and p >> 31:
                    continue  # empty DF cell: the low bits hold its distance
                if p:
                    cx, cy, cz = idx & ((1 << wx) - 1), (idx >> wx) & ((1 << wy) - 1), idx >> (wx + wy)
                    walk(d + 1, p + rb(d + 1), (corner[0] + (cx << cs), corner[1] + (cy << cs), corner[2] + (cz << cs)))
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
                child = int(W[base + 2 * rank]) + rb(d + 1)
                assert int(W[base + 2 * rank + 1]) == int(W[child]), "descriptor mask differs from the child's"
                walk(d + 1, child, c)
            else:
                walk(d + 1, int(W[base + rank]) + rb(d + 1), c)

    walk(0, root, (0, 0, 0))
    out.sort(key=lambda v: (v[2], v[1], v[0]))
    return out


def df_grids(info, words):
    """Every DF grid of the buffer: list of (kind, dims (nx, ny, nz), occupied[z, y, x], dist[z, y, x]).

    kind "D": a pointer grid (distance in cells); "E": the block grid of a last DF level
    (distance in blocks)."""
    W = [int(v) for v in words] if len(words) < 200000 else words
    D, nlev = _depths(info)
    grids = []
    regions = info.get("depth_buffers", False)
    root = int(W[0])
    if root == 0:
        return grids
    rb = (lambda d: info["depth_offset"][d] - 16 if regions and d < len(D) else 0)
    root += rb(0)

    def cells(d, ptr):
        k, kind, j, L, cs, w = D[d]
        if kind in ("D", "R"):
            dims = (1 << w[0], 1 << w[1], 1 << w[2])
            vals = np.array([int(W[ptr + i]) for i in range(dims[0] * dims[1] * dims[2])], dtype=np.uint64)
            if kind == "D":
                occ = (vals >> np.uint64(31)) == 0
                dist = np.where(occ, 0, vals & np.uint64(0x7FFFFFFF))
                grids.append(("D", dims, occ.reshape(dims[::-1]), dist.reshape(dims[::-1]).astype(np.int64)))
                kids = [int(v) for v in vals[occ]]
            else:
                kids = [int(v) for v in vals if v]
            if d + 1 < len(D) and D[d + 1][1] in ("R", "D", "B", "E"):
                for c in kids:
                    cells(d + 1, c + rb(d + 1))
            elif d + 1 < len(D):
                # octree below: DF grids deeper than an octree are not listed
                pass
        elif kind == "E":
            b = min(2, min(w))
            dims = (1 << (w[0] - b), 1 << (w[1] - b), 1 << (w[2] - b))
            nb = dims[0] * dims[1] * dims[2]
            q = np.array([int(W[ptr + i]) for i in range(4 * nb)], dtype=np.uint64).reshape(nb, 4)
            occ = (q[:, 0] | q[:, 1]) != 0
            grids.append(("E", dims, occ.reshape(dims[::-1]), q[:, 2].astype(np.int64).reshape(dims[::-1])))
            assert np.all(q[:, 3] == 0)

    cells(0, root)
    return grids


def decode_codes(info, words, morton_encode):
    v = decode(info, words)
    if not v:
        return np.zeros(0, np.uint64)
    return np.sort(morton_encode(np.array(v, dtype=np.int32)))
