"""Oracle values at sampled atoms of large periodic cells.

E_i depends only on the atoms within rcut of atom i, and the force on atom k
only on the energies of k and of the atoms within rcut of k.  So the oracle
can evaluate a sampled atom on an open cluster cut out of the cell around it:
all atoms within rcut (energy) or 2 rcut (force) of it, unwrapped by the
minimum image.  That is the same definition evaluated on the same
neighborhoods; it needs box edges above twice the cut radius, so that every
atom appears once.  A CPU test checks the cut-outs against the oracle on the
whole cell.
"""
import numpy as np

import oracle


class LocalSampler:
    def __init__(self, cfg, params, table, x, box, types=None):
        self.cfg, self.params, self.table = cfg, params, table
        self.types = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.L = np.diag(np.asarray(box, dtype=np.float64).reshape(3, 3)).copy()
        rc = cfg["rcut"]
        self.radius = 2.0 * rc + 0.5
        if np.any(self.L <= 2.0 * self.radius):
            raise ValueError("box edges must exceed 4 rcut + 1 for force cut-outs")
        # bins of edge >= radius: the 27 around an atom hold every atom within radius
        self.nb = np.floor(self.L / self.radius).astype(int)
        w = self.x - self.L * np.floor(self.x / self.L)
        c = np.minimum((w / (self.L / self.nb)).astype(int), self.nb - 1)
        self.cid = (c[:, 0] * self.nb[1] + c[:, 1]) * self.nb[2] + c[:, 2]
        self.order = np.argsort(self.cid, kind="stable")
        self.start = np.searchsorted(self.cid[self.order], np.arange(self.nb.prod() + 1))
        self.c3 = c

    def _cut(self, k, radius):
        ck = self.c3[k]
        idx = []
        for d0 in (-1, 0, 1):
            for d1 in (-1, 0, 1):
                for d2 in (-1, 0, 1):
                    c = (ck + (d0, d1, d2)) % self.nb
                    b = (c[0] * self.nb[1] + c[1]) * self.nb[2] + c[2]
                    idx.append(self.order[self.start[b]:self.start[b + 1]])
        idx = np.unique(np.concatenate(idx))
        d = self.x[idx] - self.x[k]
        d -= self.L * np.round(d / self.L)
        r = np.sqrt(np.sum(d * d, axis=1))
        keep = r < radius
        idx, d, r = idx[keep], d[keep], r[keep]
        return idx, self.x[k] + d, r

    def energy(self, k):
        idx, c, _ = self._cut(k, self.cfg["rcut"] + 0.5)
        pos = int(np.nonzero(idx == k)[0][0])
        return oracle.evaluate(self.cfg, self.params, c, None, table=self.table, centers=np.array([pos], np.int32),
                               forces=False, types=self._types(idx))["e_atom"][0]

    def _types(self, idx):
        return None if self.types is None else self.types[idx]

    def force(self, k):
        idx, c, r = self._cut(k, self.radius)
        pos = int(np.nonzero(idx == k)[0][0])
        cen = np.nonzero(r < self.cfg["rcut"])[0].astype(np.int32)
        return oracle.evaluate(self.cfg, self.params, c, None, table=self.table, centers=cen,
                               types=self._types(idx))["F"][pos]
