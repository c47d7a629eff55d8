"""Test helpers: turn the oracle tree's per-group lists into the CSR form.

Groups are arbitrary sets of original particle ids; the CSR form wants each
group to be a contiguous range, so particles are renumbered in group order.
Cells are numbered in the oracle tree's preorder and appear as n + cell.
"""
import numpy as np

from oracle import tree as otree


def o3_csr(tr, pos, groups, theta, **walk_kw):
    n = len(pos)
    order = np.concatenate(groups).astype(np.int64)
    assert len(order) == n and len(np.unique(order)) == n
    inv = np.empty(n, np.int64)
    inv[order] = np.arange(n)
    cell_no = {id(c): k for k, c in enumerate(tr.cells)}
    group_off = np.zeros(len(groups) + 1, np.int64)
    group_off[1:] = np.cumsum([len(g) for g in groups])
    lists, n_cellent, acc_cells = [], [], []
    for g in groups:
        cells, parts = otree.walk(tr, pos, g, theta, **walk_kw)
        ent = [n + cell_no[id(c)] for c in cells] + sorted(int(inv[p]) for p in parts)
        lists.append(ent)
        n_cellent.append(len(cells))
        acc_cells.append(cells)
    list_off = np.zeros(len(groups) + 1, np.int64)
    list_off[1:] = np.cumsum([len(l) for l in lists])
    list_idx = np.array([e for l in lists for e in l], np.int64)
    cell_com = np.array([c.com for c in tr.cells])
    cell_mass = np.array([c.M for c in tr.cells])
    return dict(order=order, group_off=group_off, list_off=list_off, list_idx=list_idx,
                n_cellent=np.array(n_cellent, np.int64), cell_com=cell_com,
                cell_mass=cell_mass, accepted=acc_cells)
