"""Plain FP64 octree, cell moments and group tree walk -- TEST INFRASTRUCTURE ONLY.

An independent, slow, recursive implementation used to check the production
host tree and walk.  It shares nothing with the product library.

Tree (Sec. 2 and 3.2 of the paper):
  * the root is the cube enclosing all particles: centre at the bounding-box
    centre, side = the largest bounding-box extent (no padding);
  * a cell is split into its 8 octants; a coordinate >= the cell centre goes
    to the upper half;
  * a cell with at most ``n_crit`` particles (or at depth ``max_level``) is a
    leaf.  The paper says both "less than" and "maximum number"; the reading
    taken is "at most n_crit".

Cell moments (Sec. 2.2, 3.3): total mass M, centre of mass, side l, offset
s = |COM - geometric centre|, b_max = the largest particle distance from the
COM, and the second-moment tensor S = sum m (x - COM)(x - COM)^T, whose trace
is the B2 of Eq. (2).

Walk (Sec. 2.1 rules, Sec. 3.4 vectorised groups): for a group of target
particles with bounding box [lo, hi], d_min is the distance from a cell's COM
to that box (0 inside).  Two acceptance criteria are provided:
  * 'bh'  : accept iff d_min > l / theta + s   (Barnes-Hut with the COM offset)
  * 'sw'  : accept iff d_min > r_b with r_b from Eq. (1),
            r_b = b_max/2 + sqrt(b_max^2/4 + sqrt(3 B2 / Delta)),
            and r_b = 2 * root side for cells heavier than m_limit (Sec. 3.3).
An accepted cell is one list entry; an opened leaf contributes its particles.

Near cells (the cells a learned correction is applied to; not in the paper):
the accepted cells whose side is at least ``ratio`` times the distance from
their COM to the centre of the group's bounding box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cell:
    idx: np.ndarray            # original particle ids inside the cell
    level: int
    ijk: tuple                 # integer cube coordinates at this level
    centre: np.ndarray
    side: float
    children: list = field(default_factory=list)
    M: float = 0.0
    com: np.ndarray = None
    s: float = 0.0
    b_max: float = 0.0
    S: np.ndarray = None

    @property
    def leaf(self):
        return not self.children

    @property
    def key(self):
        """Identity of the cell as a geometric cube: (level, i, j, k)."""
        return (self.level,) + tuple(int(v) for v in self.ijk)


@dataclass
class Tree:
    root: Cell
    cells: list                # all cells, preorder
    root_side: float
    root_lo: np.ndarray


def _moments(cell: Cell, pos: np.ndarray, mass: np.ndarray):
    p = pos[cell.idx]
    m = mass[cell.idx]
    cell.M = float(m.sum())
    cell.com = (m[:, None] * p).sum(axis=0) / cell.M
    r = p - cell.com
    cell.S = (m[:, None, None] * r[:, :, None] * r[:, None, :]).sum(axis=0)
    cell.b_max = float(np.sqrt((r * r).sum(axis=1)).max())
    cell.s = float(np.linalg.norm(cell.com - cell.centre))


def build(pos: np.ndarray, mass: np.ndarray, n_crit: int = 16, max_level: int = 21) -> Tree:
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    lo = pos.min(axis=0)
    hi = pos.max(axis=0)
    centre = 0.5 * (lo + hi)
    side = float((hi - lo).max())
    if side == 0.0:
        side = 1.0
    cells: list = []

    def make(idx, level, ijk, c, sd):
        cell = Cell(idx=idx, level=level, ijk=ijk, centre=c, side=sd)
        _moments(cell, pos, mass)
        cells.append(cell)
        if len(idx) > n_crit and level < max_level:
            p = pos[idx]
            upper = p >= c
            octant = upper[:, 0] * 1 + upper[:, 1] * 2 + upper[:, 2] * 4
            for o in range(8):
                sub = idx[octant == o]
                if len(sub) == 0:
                    continue
                bits = np.array([(o >> 0) & 1, (o >> 1) & 1, (o >> 2) & 1])
                cc = c + (bits - 0.5) * (sd / 2.0)
                cijk = tuple(2 * np.array(ijk) + bits)
                cell.children.append(make(sub, level + 1, cijk, cc, sd / 2.0))
        return cell

    root = make(np.arange(len(pos)), 0, (0, 0, 0), centre, side)
    return Tree(root=root, cells=cells, root_side=side, root_lo=centre - side / 2)


def box_distance(point: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> float:
    """Euclidean distance from a point to an axis-aligned box (0 inside)."""
    d = np.maximum(0.0, np.maximum(lo - point, point - hi))
    return float(np.sqrt((d * d).sum()))


def sw_radius(b_max: float, B2: float, delta: float) -> float:
    """Bounding radius of the absolute MAC, Eq. (1)."""
    return b_max / 2.0 + math.sqrt(b_max * b_max / 4.0 + math.sqrt(3.0 * B2 / delta))


def walk(tree: Tree, pos: np.ndarray, group_ids: np.ndarray, theta: float = 0.5,
         mac: str = "bh", delta: float = 0.01, m_limit: float = math.inf):
    """Interaction list of one group.

    Returns (cells, particles): the accepted cells (Cell objects) and the
    original ids of particles from opened leaves, both in tree preorder.
    """
    p = np.asarray(pos, dtype=np.float64)[group_ids]
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    out_cells: list = []
    out_parts: list = []

    def accept(cell: Cell) -> bool:
        d = box_distance(cell.com, lo, hi)
        if mac == "bh":
            if theta <= 0.0:
                return False
            return d > cell.side / theta + cell.s
        if mac == "sw":
            if cell.M > m_limit:
                rb = 2.0 * tree.root_side
            else:
                rb = sw_radius(cell.b_max, float(np.trace(cell.S)), delta)
            return d > rb
        raise ValueError(mac)

    def visit(cell: Cell):
        if accept(cell):
            out_cells.append(cell)
            return
        if cell.leaf:
            out_parts.extend(int(i) for i in cell.idx)
            return
        for ch in cell.children:
            visit(ch)

    visit(tree.root)
    return out_cells, out_parts


def cell_groups(tree: Tree, g_max: int) -> list:
    """Groups as the maximal cells holding at most g_max particles."""
    out = []

    def visit(cell: Cell):
        if len(cell.idx) <= g_max:
            out.append(np.sort(cell.idx))
            return
        if cell.leaf:
            # a leaf at the depth cap can exceed g_max: split it in id order
            ids = np.sort(cell.idx)
            for k in range(0, len(ids), g_max):
                out.append(ids[k:k + g_max])
            return
        for ch in cell.children:
            visit(ch)

    visit(tree.root)
    return out


def near_cells(cells: list, pos: np.ndarray, group_ids: np.ndarray, ratio: float) -> list:
    """The accepted cells of a group that are near in the sense above:
    side >= ratio * |COM - (lo + hi) / 2| with [lo, hi] the group's
    bounding box, in FP64."""
    p = np.asarray(pos, dtype=np.float64)[group_ids]
    centre = 0.5 * (p.min(axis=0) + p.max(axis=0))
    return [c for c in cells if c.side >= ratio * float(np.linalg.norm(c.com - centre))]
