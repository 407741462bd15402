"""Step 1-2 (tile intersection) and Step 2 (depth sorting), replayed in float32
(oracle; test infrastructure).

Tiles are 16x16 pixels (Sec. 2.1, footnote on tiles).  A Gaussian is listed in
every tile that meets its padded pixel rectangle.  The rectangle is the
bounding box of the ellipse on which alpha~ = 1/255, i.e.
d^T M d <= 2 ln(255 o), whose half-widths are e_x = sqrt(2 ln(255 o) Sigma'_xx)
and e_y likewise, widened by one pixel on each side:

    x_lo = floor((u - e_x) - 1.5),  x_hi = ceil((u + e_x) + 0.5)

in float32, operations in that order (pixel i samples at i + 0.5, so pixel i
lies in the box when u - e_x - 0.5 <= i <= u + e_x - 0.5).  Empty when
x_hi < 0 or x_lo > W - 1; otherwise clamped to [0, W - 1] and divided by 16.

The replay takes the float32 (u, v, e_x, e_y, z) that the kernel under test
produced for each Gaussian, so the integer lists can be compared bit for bit;
those float32 stage values are compared separately, within tolerance, against
the float64 projection.

Order inside a tile: ascending (bits of the float32 depth, Gaussian id), i.e.
front to back with ties broken by index (Step 2).

Pins: tests/test_oracle_pins.py (lists against a per-(tile, Gaussian) loop
with Python's sorted() on tuples; conservativeness against the float64
fragment set).
"""
import numpy as np

TILE = 16


def tile_rects(u, v, ex, ey, valid, width, height, tile_w=TILE, tile_h=TILE):
    """Per-Gaussian inclusive tile rectangle (tx0, ty0, tx1, ty1); empty rows
    get tx1 < tx0.  Tiles are tile_w x tile_h pixels (16 x 16, or larger for a
    frame rendered with one sample per block of pixels)."""
    f = np.float32
    u, v, ex, ey = (np.asarray(t, dtype=np.float32) for t in (u, v, ex, ey))
    lo_x = np.floor((u - ex) - f(1.5))
    hi_x = np.ceil((u + ex) + f(0.5))
    lo_y = np.floor((v - ey) - f(1.5))
    hi_y = np.ceil((v + ey) + f(0.5))
    empty = ((hi_x < 0) | (lo_x > width - 1) | (hi_y < 0) | (lo_y > height - 1)
             | ~np.asarray(valid, dtype=bool))
    with np.errstate(invalid="ignore"):
        i0 = np.clip(lo_x, 0, width - 1)
        i1 = np.clip(hi_x, 0, width - 1)
        j0 = np.clip(lo_y, 0, height - 1)
        j1 = np.clip(hi_y, 0, height - 1)
    i0, i1, j0, j1 = (np.nan_to_num(t).astype(np.int64) for t in (i0, i1, j0, j1))
    tx0, tx1, ty0, ty1 = i0 // tile_w, i1 // tile_w, j0 // tile_h, j1 // tile_h
    tx1 = np.where(empty, tx0 - 1, tx1)
    return tx0, ty0, tx1, ty1


def tile_lists(u, v, ex, ey, z, valid, width, height, tile_w=TILE, tile_h=TILE):
    """Sorted tile lists: (ranges [T,2] int64, ids [P] int64), tiles in
    row-major order."""
    tiles_x = (width + tile_w - 1) // tile_w
    tiles_y = (height + tile_h - 1) // tile_h
    tx0, ty0, tx1, ty1 = tile_rects(u, v, ex, ey, valid, width, height, tile_w, tile_h)
    nx = np.maximum(tx1 - tx0 + 1, 0)
    ny = np.where(nx > 0, np.maximum(ty1 - ty0 + 1, 0), 0)
    cnt = nx * ny
    gid = np.repeat(np.arange(len(cnt)), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(cnt.sum()) - start
    nxg = nx[gid]
    tx = tx0[gid] + k % np.maximum(nxg, 1)
    ty = ty0[gid] + k // np.maximum(nxg, 1)
    tile = ty * tiles_x + tx
    zbits = np.asarray(z, dtype=np.float32).view(np.uint32).astype(np.int64)[gid]
    order = np.lexsort((gid, zbits, tile))
    tile, gid = tile[order], gid[order]
    counts = np.bincount(tile, minlength=tiles_x * tiles_y)
    ends = np.cumsum(counts)
    ranges = np.stack([ends - counts, ends], 1)
    return ranges, gid


def pair_change(rect_ref, rect_cur, skip=None):
    """Change of the tile-Gaussian intersections between two sets of tile
    rectangles (the ratio of Sec. 4.1 that sets the next pruning interval),
    by brute force over explicit tile sets: returns (pairs in exactly one of
    the two rectangles, pairs of rect_ref), summed over the Gaussians i with
    skip[i] false.  Rectangles are rows (x0, y0, x1, y1), inclusive, empty
    when x1 < x0 or y1 < y0."""
    def tiles(r):
        x0, y0, x1, y1 = (int(t) for t in r)
        return {(x, y) for x in range(x0, x1 + 1) for y in range(y0, y1 + 1)}

    changed = ref = 0
    for i, (a, b) in enumerate(zip(rect_ref, rect_cur)):
        if skip is not None and skip[i]:
            continue
        ta, tb = tiles(a), tiles(b)
        changed += len(ta ^ tb)
        ref += len(ta)
    return changed, ref

