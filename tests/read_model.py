"""Reference set of the format words a walk must read for one ray (test only).

B_ray, the numerator of every roofline figure, is the counting kernel's set of distinct
format words (and 64-byte sectors) each ray reads. This module derives the set the
traversal of the paper (Sec. 4.2) has to read, on its own: it walks the volume's cells
level by level in order of entry time, with plane times computed as the walk defines them
(fp32, 1/d correctly rounded, (p - o) * (1/d) never fused), decides occupancy from the
voxel set, stops at the first occupied voxel, and maps each cell it tests or enters to the
words of the library's layout (or of the paper's layout) that hold it:

* word 0, the root pointer, and the root node's header words;
* a Raw pointer-grid cell: its one word, when tested; a brick block: its 64-bit mask
  (two words; four with a distance field), when tested; a voxel inside a block: none;
* an SVO child: its two header words, when entered; an SVDAG child: its (pointer, mask)
  descriptor, two words, when entered; a pointer to the next level's root: one word,
  then that root's header words;
* a distance-field cell within the reach of the last empty cell read is not read (the
  skip rule of the walk: reach = that cell's stored distance, counted in L1 cells);
* the paper's layout: RGBA words per voxel, (term, distance) pairs per DF cell, one
  pointer per SVDAG child and a leaf word holding the next level's pointer.

It shares no code with the library or the oracle; only the layout's documented structure
(node headers, ranks, x-fastest cells) locates words.
"""
import numpy as np

F32 = np.float32
INF = F32(np.inf)
DF_EMPTY = 0x80000000


def _fmax(a, b):
    return b if a < b else a


def _fmin(a, b):
    return b if b < a else a


class Ray:
    """Setup of the walk: 1/d in fp32; an axis is parallel iff 1/d is not finite."""

    def __init__(self, r, ext_log2):
        o = [F32(r[0]), F32(r[1]), F32(r[2])]
        d = [F32(r[4]), F32(r[5]), F32(r[6])]
        self.o, self.d = o, d
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            self.inv = [F32(1.0) / d[a] for a in range(3)]
        self.par = [not np.isfinite(self.inv[a]) for a in range(3)]
        self.ok = all(np.isfinite(o[a]) and np.isfinite(d[a]) for a in range(3)) and not all(self.par)
        for a in range(3):
            if self.par[a] and not (F32(0) <= o[a] < F32(1 << ext_log2[a])):
                self.ok = False
        self.t0, self.t1 = F32(r[3]), F32(r[7])
        if self.ok:
            first, tn, tf = True, F32(0), F32(0)
            for a in range(3):
                if self.par[a]:
                    continue
                N = 1 << ext_log2[a]
                ne, fa = self.T(a, N if d[a] < 0 else 0), self.T(a, 0 if d[a] < 0 else N)
                tn = ne if first else _fmax(tn, ne)
                tf = fa if first else _fmin(tf, fa)
                first = False
            self.t0, self.t1 = _fmax(self.t0, tn), _fmin(self.t1, tf)
            self.ok = bool(self.t0 < self.t1)

    def T(self, a, p):
        with np.errstate(over="ignore", invalid="ignore"):
            return F32(F32(F32(p) - self.o[a]) * self.inv[a])

    def interval(self, c, s):
        """Visit interval [e, x) of the cube at corner c with side s, clipped to [t0, t1)."""
        e, x = self.t0, self.t1
        for a in range(3):
            if self.par[a]:
                if not (c[a] <= np.floor(self.o[a]) < c[a] + s):
                    return None
                continue
            lo, hi = self.T(a, c[a]), self.T(a, c[a] + s)
            near, far = (hi, lo) if self.d[a] < 0 else (lo, hi)
            e, x = _fmax(e, near), _fmin(x, far)
        return (e, x) if e < x else None


def _levels(info):
    """Per level: (kind R/D/S/G, exponents, DF cap); sub[k]: log2 side of a level-k sub-volume."""
    kinds, exps, maxd = info["kinds"], info["level_exp"], info["level_maxdist"]
    n = len(kinds)
    sub = [0] * (n + 1)
    for k in range(n - 1, 0, -1):
        sub[k] = sub[k + 1] + exps[k][0]
    return [(kinds[k], exps[k], maxd[k]) for k in range(n)], sub


class Model:
    def __init__(self, info, words, voxels):
        self.info = info
        self.W = [int(v) for v in words]
        self.paper = bool(info["paper_layout"])
        self.lv, self.sub = _levels(info)
        self.ext = info["extent_log2"]
        self.occ = {}
        v = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
        for k in range(max(self.ext) + 1):
            self.occ[k] = set(map(tuple, (v >> k).tolist()))

    def occupied(self, c, log2s):
        return (c[0] >> log2s, c[1] >> log2s, c[2] >> log2s) in self.occ[log2s]

    def reads(self, r):
        """(set of word indices read, hit voxel or None) for the ray r (8 floats)."""
        R = Ray(r, self.ext)
        out = set()
        if not R.ok:
            return out, None
        out.add(0)
        root = self.W[0]
        if root == 0:
            return out, None
        hit = self._level(R, 0, root, (0, 0, 0), out)
        return out, hit

    # A sub-volume of level k, rooted at pointer ptr, corner c.
    def _level(self, R, k, ptr, c, out):
        kind, e, maxd = self.lv[k]
        last = k == len(self.lv) - 1
        cs = self.sub[k + 1]
        if kind in "RD":
            if last and not self.paper:
                return self._brick(R, k, ptr, c, out)
            return self._grid(R, k, ptr, c, out, cs, last)
        return self._octree(R, k, ptr, c, out)

    def _cells(self, R, c, w, cs):
        """Cells of a grid of 2^w[a] cells of side 2^cs at corner c that the ray visits, in
        entry order: (lin, corner, e, x)."""
        cells = []
        for lin in range(1 << (w[0] + w[1] + w[2])):
            ix = (lin & ((1 << w[0]) - 1), (lin >> w[0]) & ((1 << w[1]) - 1), lin >> (w[0] + w[1]))
            cc = tuple(c[a] + (ix[a] << cs) for a in range(3))
            iv = R.interval(cc, 1 << cs)
            if iv is not None:
                cells.append((lin, cc, iv[0], iv[1]))
        cells.sort(key=lambda q: q[2])
        return cells

    def _grid(self, R, k, base, c, out, cs, last):
        """A Raw or DF grid read cell by cell (a pointer-grid level, or any Raw/DF level of
        the paper's layout)."""
        kind, w, maxd = self.lv[k]
        df = kind == "D"
        stride = 2 if (self.paper and df) else 1
        anchor, reach = None, 0
        for lin, cc, e, x in self._cells(R, c, w, cs):
            if df and reach and sum(abs(cc[a] - anchor[a]) for a in range(3)) >> cs < reach:
                assert not self.occupied(cc, cs), "a skipped cell is occupied"
                continue
            out.update(range(base + stride * lin, base + stride * lin + stride))
            occ = self.occupied(cc, cs)
            if df and not occ:
                word = self.W[base + stride * lin + (1 if self.paper else 0)]
                anchor, reach = cc, (word if self.paper else word & ~DF_EMPTY)
                continue
            if not occ:
                continue
            if last:
                return cc
            child = self.W[base + stride * lin]
            hit = self._enter(R, k + 1, child, cc, out)
            if hit is not None:
                return hit
            reach = 0
        return None

    def _brick(self, R, k, base, c, out):
        """The last Raw/DF level of the library's layout: blocks of side 2^b (two words of
        mask each, four with a distance field), then the voxels of a block (registers)."""
        kind, e, maxd = self.lv[k]
        b = min(2, min(e))
        blk = [e[a] - b for a in range(3)]
        if sum(blk) == 0:  # a one-block brick: its mask is read on entry
            out.update((base, base + 1))
            return self._voxels(R, c, b)
        df = kind == "D"
        st = 4 if df else 2
        anchor, reach = None, 0
        for lin, cc, e_, x_ in self._cells(R, c, blk, b):
            if df and reach and sum(abs(cc[a] - anchor[a]) for a in range(3)) >> b < reach:
                assert not self.occupied(cc, b), "a skipped block is occupied"
                continue
            out.update(range(base + st * lin, base + st * lin + st))
            if not self.occupied(cc, b):
                if df:
                    anchor, reach = cc, self.W[base + st * lin + 2]
                continue
            hit = self._voxels(R, cc, b)
            if hit is not None:
                return hit
            reach = 0
        return None

    def _voxels(self, R, c, b):
        for lin, cc, e, x in self._cells(R, c, (b, b, b), 0):
            if self.occupied(cc, 0):
                return cc
        return None

    def _enter(self, R, k, ptr, c, out):
        """Enter the root node of level k at pointer ptr (its header words are read)."""
        return self._level(R, k, ptr, c, out)

    def _octree(self, R, k, ptr, c, out):
        kind, e, maxd = self.lv[k]
        L = e[0]
        last = k == len(self.lv) - 1
        W = self.W
        # the level's root node header
        if kind == "S":
            out.update((ptr, ptr + 1))
            base, valid = W[ptr], W[ptr + 1] & 0xFF
        else:
            out.add(ptr)
            base, valid = ptr + 1, W[ptr] & 0xFF
        return self._node(R, k, 0, L, base, valid, c, out, last)

    def _node(self, R, k, j, L, base, valid, c, out, last):
        kind = self.lv[k][0]
        cs = self.sub[k + 1] + (L - 1 - j)
        W = self.W
        for o, cc, e, x in self._cells(R, c, (1, 1, 1), cs):
            if not self.occupied(cc, cs):
                continue
            assert (valid >> o) & 1, "the node mask disagrees with the voxels"
            rank = bin(valid & ((1 << o) - 1)).count("1")
            if j == L - 1:
                if last:
                    return cc
                if self.paper and kind == "S":  # the child's first word points to the next level
                    out.add(base + 2 * rank)
                    child = W[base + 2 * rank]
                elif self.paper:  # a pointer to a leaf word that holds the next level's pointer
                    out.add(base + rank)
                    out.add(W[base + rank])
                    child = W[W[base + rank]]
                else:
                    out.add(base + rank)
                    child = W[base + rank]
                hit = self._enter(R, k + 1, child, cc, out)
            elif kind == "S":
                ch = base + 2 * rank
                out.update((ch, ch + 1))
                hit = self._node(R, k, j + 1, L, W[ch], W[ch + 1] & 0xFF, cc, out, last)
            elif self.paper:
                ch = W[base + rank]
                out.add(base + rank)
                out.add(ch)
                hit = self._node(R, k, j + 1, L, ch + 1, W[ch] & 0xFF, cc, out, last)
            else:  # (child pointer, copy of the child's mask word)
                out.update((base + 2 * rank, base + 2 * rank + 1))
                ch = W[base + 2 * rank]
                hit = self._node(R, k, j + 1, L, ch + 1, W[base + 2 * rank + 1] & 0xFF, cc, out, last)
            if hit is not None:
                return hit
        return None
