"""Index arithmetic of the point tiles' pattern pass, emulated on the CPU.

The tile kernel places the mark of a structural pair (j, l) at l's position
in j's walk of cells (the 5^(d-1) rows of cells within two of j's cell):
the walk-table row of j's cell is looked up by the slot of that cell among
the tile cell's 3^d neighbours, and the row by the cells' offset in y (and
z).  These checks rebuild grids, windows (active centres whose ball reaches
the cell) and walk tables with the kernel's formulas for small 2D and 3D
configurations, boundary cells included, and require every slot and every
position of every window pair to fall inside its table and its row.  A
slot formula with a z term in 2D fails them.
"""
import numpy as np
import pytest

import synthdata as sd


def grid_of(ctr, rho):
    dim = ctr.shape[0]
    cs = rho * (1 + 1e-6)
    lo_c, hi_c = ctr.min(1), ctr.max(1)
    g = np.ones(3, int)
    glo = np.zeros(3)
    for k in range(dim):
        glo[k] = lo_c[k] - 1.5 * cs
        g[k] = int(np.ceil(((hi_c[k] - lo_c[k]) + 3 * cs) / cs)) + 1
    return cs, g, glo


def cells_of(x, cs, g, glo):
    dim = x.shape[0]
    c = np.zeros((3, x.shape[1]), np.int64)
    inb = np.ones(x.shape[1], bool)
    for d in range(dim):
        c[d] = np.floor((x[d] - glo[d]) / cs).astype(np.int64)
        inb &= (c[d] >= 0) & (c[d] < g[d])
    return c, inb


def walk(c, reach, g, dim):
    w = 2 * reach + 1
    rows = []
    for k in range(w if dim == 2 else w * w):
        y = c[1] + k % w - reach
        z = c[2] + k // w - reach if dim == 3 else 0
        if y < 0 or y >= g[1] or z < 0 or z >= g[2]:
            rows.append(None)
            continue
        x0, x1 = max(c[0] - reach, 0), min(c[0] + reach, g[0] - 1)
        rows.append((x0 + g[0] * (y + g[1] * z), x1 + g[0] * (y + g[1] * z)))
    return rows


def slot(dc, dim):
    """The kernel's slot of a neighbour cell at offset dc from the tile's."""
    return (dc[0] + 1) + 3 * (dc[1] + 1) + (9 * (dc[2] + 1) if dim == 3 else 0)


def walk_row(ca, cb, dim):
    return (cb[1] - ca[1] + 2) + (5 * (cb[2] - ca[2] + 2) if dim == 3 else 0)


@pytest.mark.parametrize("dim,g_ctr,rho_cells,n", [(2, 12, 2.2, 3000), (3, 6, 1.6, 3000)])
def test_pattern_slots_and_positions_in_range(dim, g_ctr, rho_cells, n):
    rng = np.random.default_rng(7 + dim)
    ctr = sd.grid_centers(g_ctr, dim)
    rho = rho_cells / (g_ctr - 1)
    pts = np.concatenate([rng.random((dim, n // 2)),
                          sd.gaussian_mixture_points(rng, n - n // 2, dim, 3)], axis=1)
    m = ctr.shape[1]
    cs, g, glo = grid_of(ctr, rho)
    ncell = int(np.prod(g))
    cc, _ = cells_of(ctr, cs, g, glo)
    cid = cc[0] + g[0] * cc[1] + g[0] * g[1] * cc[2]
    order = np.argsort(cid, kind="stable")
    spos = np.empty(m, np.int64)
    spos[order] = np.arange(m)
    ccs = np.searchsorted(cid[order], np.arange(ncell + 2))
    d2 = ((pts[:, :, None] - ctr[:, None, :]) ** 2).sum(0)
    active = (d2 < rho * rho).sum(0) >= 1
    pc, pin = cells_of(pts, cs, g, glo)
    pcid = (pc[0] + g[0] * pc[1] + g[0] * g[1] * pc[2])[pin]
    R = 5 if dim == 2 else 25
    NC = 9 if dim == 2 else 27

    def decode(c):
        return np.array([c % g[0], (c // g[0]) % g[1], c // (g[0] * g[1]) if dim == 3 else 0])

    def table(cell):
        t, off = [], 0
        for r in walk(decode(cell), 2, g, dim):
            if r is None:
                t.append((0, off))
                continue
            a, b = ccs[r[0]], ccs[r[1] + 1]
            t.append((a, off))
            off += b - a
        return np.array(t), off

    checked = 0
    for cell in np.unique(pcid):
        c = decode(cell)
        lo = glo[:dim] + c[:dim] * cs - 1e-6 * cs
        hi = glo[:dim] + (c[:dim] + 1) * cs + 1e-6 * cs
        win = []
        for r in walk(c, 1, g, dim):
            if r is None:
                continue
            for i in range(ccs[r[0]], ccs[r[1] + 1]):
                l = order[i]
                x = ctr[:dim, l]
                t = np.where(x < lo, lo - x, np.where(x > hi, x - hi, 0.0))
                if active[l] and np.sum(t * t) <= rho * rho * (1 + 1e-9):
                    win.append(l)
        if not win:
            continue
        win = np.array(win)
        dc = cc[:, win] - c[:, None]
        assert np.all(np.abs(dc) <= 1)
        slots = np.array([slot(dc[:, a], dim) for a in range(len(win))])
        assert slots.min() >= 0 and slots.max() < NC
        # the tile's table rows, loaded per slot as the kernel does
        tt = np.zeros((NC, R, 2), np.int64)
        for sl in range(NC):
            cn = np.array([c[0] + sl % 3 - 1, c[1] + (sl // 3) % 3 - 1,
                           c[2] + sl // 9 - 1 if dim == 3 else 0])
            if np.all(cn[:dim] >= 0) and np.all(cn[:dim] < g[:dim]):
                tt[sl] = table(int(cn[0] + g[0] * cn[1] + g[0] * g[1] * cn[2]))[0]
        lens = np.array([table(int(x))[1] for x in cid[win]])
        for a in range(len(win)):
            for b in range(len(win)):
                row = walk_row(dc[:, a], dc[:, b], dim)
                assert 0 <= row < R
                st, off = tt[slots[a], row]
                p = off + spos[win[b]] - st
                assert 0 <= p < lens[a], (cell, a, b, p, lens[a])
                checked += 1
    assert checked > 1000


def test_slot_formula_has_no_z_term_in_2d():
    # in 2D every neighbour offset maps into the 9 loaded rows
    s = {slot((dx, dy, 0), 2) for dx in (-1, 0, 1) for dy in (-1, 0, 1)}
    assert s == set(range(9))
    s3 = {slot((dx, dy, dz), 3) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)}
    assert s3 == set(range(27))
