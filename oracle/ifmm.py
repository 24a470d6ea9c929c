"""Oracle: the inverse fast multipole method (IFMM) on the completed
double-layer matrix, in plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (tests, the entry-point smoke check, the CPU
baseline of the benchmark).

The IFMM is an approximation (Section 3: tunable accuracy eps), so it is never
the parity target of a solve: the GPU solver is compared with the dense LU
solution.  This module exists to pin the method itself: it must become a
direct solver as eps -> 0, be exact when the tree has no well-separated pair,
and its error must follow eps.  It takes the steps of Section 3 in order:

1. H^2 representation (Section 3.1, equation "A_H"): a uniform quadtree;
   near-field blocks S (self and neighbours at the leaves); far field through
   nested bases built from Chebyshev interpolation with n nodes per direction,
   reduced by an SVD of the interpolated kernel (Section 4, black-box
   construction).  Each box keeps one orthonormal basis W used on both sides
   (U = V = W; a reading, see the design notes).
2. Extended sparsification (Section 3.2): per box the unknowns sigma_b
   (here x_b), the local coefficients z_b and the multipole coefficients
   y_b = W_b^T x_b, with rows R_b (original equations), Y_b (definition of
   y_b) and Z_b (local expansion z_b = sum T y + transfer from the parent).
3. Elimination (Section 3.3), level by level from the leaves: for box i the
   pivot rows (R_i, Y_i) eliminate (x_i, z_i).  The Schur complement creates
   fill-ins between the neighbours of i; those between neighbours are added
   to the near field, those between well-separated boxes, and those between
   x-rows and the multipole / local variables, are compressed by a truncated
   SVD at tolerance eps and redirected through augmented bases
   (recompression), so the sparsity pattern is kept.
4. After a level is eliminated the remaining (y, Z) system is the H^2 matrix
   of the parent level (equation "A_H" applied recursively); at the top the
   remaining dense system is solved directly.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import dlp

INV4PI = 1.0 / (4.0 * math.pi)


# ----------------------------------------------------------------------------
# Chebyshev interpolation
# ----------------------------------------------------------------------------

def cheb_points(n: int) -> np.ndarray:
    """Chebyshev points of the first kind on [-1, 1]."""
    return np.cos((2.0 * np.arange(n) + 1.0) * math.pi / (2.0 * n))


def cheb_interp_1d(n: int, t: np.ndarray) -> np.ndarray:
    """S_n(t, t_a) = 1/n + 2/n sum_{k=1}^{n-1} T_k(t) T_k(t_a), shape (len(t), n)."""
    t = np.asarray(t, dtype=np.float64)
    ta = cheb_points(n)
    out = np.full((t.shape[0], n), 1.0 / n)
    tk_prev, tk = np.ones_like(t), t.copy()
    ak_prev, ak = np.ones_like(ta), ta.copy()
    for _ in range(1, n):
        out += (2.0 / n) * tk[:, None] * ak[None, :]
        tk_prev, tk = tk, 2.0 * t * tk - tk_prev
        ak_prev, ak = ak, 2.0 * ta * ak - ak_prev
    return out


def cheb_interp_2d(n: int, px, py, cx: float, cy: float, h: float) -> np.ndarray:
    """Tensor Lagrange basis of the n x n Chebyshev grid of the box with
    centre (cx, cy) and side h, evaluated at points; shape (p, n*n), column
    index a*n + b for x-node a and y-node b."""
    sx = cheb_interp_1d(n, (np.asarray(px) - cx) * (2.0 / h))
    sy = cheb_interp_1d(n, (np.asarray(py) - cy) * (2.0 / h))
    return (sx[:, :, None] * sy[:, None, :]).reshape(sx.shape[0], n * n)


def grid_points(n: int, cx: float, cy: float, h: float):
    t = cheb_points(n) * (0.5 * h)
    gx = np.repeat(cx + t, n)
    gy = np.tile(cy + t, n)
    return gx, gy


# far-field kernel between Chebyshev grids: 2 target components x 7 source
# components (4 double-layer charges w n_k sigma_l, 2 Stokeslet, 1 rotlet)
NSRC = 7


def far_kernel(tx, ty, sx, sy) -> np.ndarray:
    """K[(a, t), (c, s)] for target comps a in {x, y} and source comps
    c = (DLP kl = xx, xy, yx, yy, Stokeslet x, y, rotlet)."""
    rx = tx[:, None] - sx[None, :]
    ry = ty[:, None] - sy[None, :]
    r2 = rx * rx + ry * ry
    inv4 = 1.0 / (r2 * r2)
    lg = 0.5 * np.log(r2)
    nt, ns = rx.shape
    k = np.zeros((2, nt, NSRC, ns))
    r = (rx, ry)
    for a in range(2):
        for kk in range(2):
            for ll in range(2):
                k[a, :, 2 * kk + ll, :] = r[a] * r[kk] * r[ll] * inv4 / math.pi
        for b in range(2):
            k[a, :, 4 + b, :] = INV4PI * ((-lg if a == b else 0.0) + r[a] * r[b] / r2)
    k[0, :, 6, :] = INV4PI * ry / r2
    k[1, :, 6, :] = -INV4PI * rx / r2
    return k.reshape(2 * nt, NSRC * ns)


def kernel_bases(n: int, h: float, eps: float):
    """SVD reduction of the interpolated far-field kernel (Section 4: the
    Chebyshev construction is followed by an SVD to reduce the rank).  The
    kernel blocks of the 40 relative positions of a box's interaction list
    are stacked side by side (target basis U_K, 2n^2 x rU) and on top of each
    other (source basis V_K, 7n^2 x rV); singular values below eps times the
    largest are dropped."""
    gx, gy = grid_points(n, 0.0, 0.0, h)
    blocks = []
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            if max(abs(dx), abs(dy)) < 2:
                continue
            sx, sy = grid_points(n, dx * h, dy * h, h)
            blocks.append(far_kernel(gx, gy, sx, sy))
    u, s, _ = np.linalg.svd(np.concatenate(blocks, axis=1), full_matrices=False)
    ru = int((s > eps * s[0]).sum())
    _, s2, vt = np.linalg.svd(np.concatenate(blocks, axis=0), full_matrices=False)
    rv = int((s2 > eps * s2[0]).sum())
    return u[:, :ru], vt[:rv].T


def orth_trunc(c: np.ndarray, tol: float) -> np.ndarray:
    """Orthonormal basis of the column space of c, with columns normalised
    first and singular values below tol * s_max dropped."""
    if c.shape[1] == 0 or c.shape[0] == 0:
        return np.zeros((c.shape[0], 0))
    nrm = np.linalg.norm(c, axis=0)
    keep = nrm > 0
    c = c[:, keep] / nrm[keep]
    if c.shape[1] == 0:
        return np.zeros((c.shape[0], 0))
    u, s, _ = np.linalg.svd(c, full_matrices=False)
    r = int((s > tol * s[0]).sum())
    return u[:, :r]


# ----------------------------------------------------------------------------
# Quadtree
# ----------------------------------------------------------------------------

def _morton(ix, iy):
    code = 0
    for b in range(32):
        code |= ((ix >> b) & 1) << (2 * b) | ((iy >> b) & 1) << (2 * b + 1)
    return code


class Level:
    def __init__(self, keys, h, x0, y0):
        order = sorted(range(len(keys)), key=lambda i: _morton(*keys[i]))
        self.keys = [keys[i] for i in order]
        self.index = {k: i for i, k in enumerate(self.keys)}
        self.h = h
        self.center = [(x0 + (k[0] + 0.5) * h, y0 + (k[1] + 0.5) * h) for k in self.keys]
        nb = len(self.keys)
        self.neighbors = []
        for (ix, iy) in self.keys:
            lst = [self.index[(ix + dx, iy + dy)] for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                   if (ix + dx, iy + dy) in self.index]
            self.neighbors.append(sorted(lst))
        self.parent = [None] * nb
        self.children = [[] for _ in range(nb)]
        self.ilist = [[] for _ in range(nb)]

    def __len__(self):
        return len(self.keys)


class Tree:
    """Uniform quadtree over the bounding square of the wall (Section 4:
    uniform decomposition; depth chosen from the mean leaf occupancy)."""

    def __init__(self, geom, leaf_target: int = 64, max_depth: int = 0):
        ws = geom.wall_slice
        xs = geom.x[ws] if ws.stop > ws.start else geom.x
        ys = geom.y[ws] if ws.stop > ws.start else geom.y
        allx = np.concatenate([geom.x, geom.cx])
        ally = np.concatenate([geom.y, geom.cy])
        lo_x, lo_y = min(allx.min(), xs.min()), min(ally.min(), ys.min())
        ext = max(allx.max() - lo_x, ally.max() - lo_y)
        self.size = ext * (1.0 + 1e-9) + 1e-12
        self.x0 = lo_x - 1e-12 * self.size
        self.y0 = lo_y - 1e-12 * self.size
        self.px, self.py = allx, ally   # node points then pore centres
        nn = geom.n_nodes
        depth = 1
        while True:
            h = self.size / 2 ** depth
            kx = np.floor((geom.x - self.x0) / h).astype(np.int64)
            ky = np.floor((geom.y - self.y0) / h).astype(np.int64)
            nbox = len(set(zip(kx.tolist(), ky.tolist())))
            if nn / nbox <= leaf_target or (max_depth and depth >= max_depth) or depth >= 20:
                break
            depth += 1
        self.depth = depth
        self.levels = []
        for lev in range(depth + 1):
            h = self.size / 2 ** lev
            kx = np.floor((self.px - self.x0) / h).astype(np.int64)
            ky = np.floor((self.py - self.y0) / h).astype(np.int64)
            keys = sorted(set(zip(kx.tolist(), ky.tolist())))
            self.levels.append(Level(keys, h, self.x0, self.y0))
            if lev == depth:
                self.leaf_kx, self.leaf_ky = kx, ky
        for lev in range(1, depth + 1):
            L, P = self.levels[lev], self.levels[lev - 1]
            for b, (ix, iy) in enumerate(L.keys):
                p = P.index[(ix // 2, iy // 2)]
                L.parent[b] = p
                P.children[p].append(b)
            for b, (ix, iy) in enumerate(L.keys):
                pn = P.neighbors[L.parent[b]]
                nset = set(L.neighbors[b])
                il = []
                for q in pn:
                    for c in P.children[q]:
                        if c not in nset:
                            il.append(c)
                L.ilist[b] = sorted(il)
        # root level: the finest level whose boxes are all mutual neighbours
        self.root = 0
        for lev in range(depth + 1):
            L = self.levels[lev]
            if all(len(L.neighbors[b]) == len(L) for b in range(len(L))):
                self.root = lev
        # leaf dofs: per box [x-comps of nodes | y-comps of nodes | centre dofs]
        leaf = self.levels[depth]
        self.leaf_dofs = []
        bx = [leaf.index[(int(a), int(b))] for a, b in zip(kx, ky)]
        members = [[] for _ in range(len(leaf))]
        for p, b in enumerate(bx):
            members[b].append(p)
        self.leaf_members = members
        for b in range(len(leaf)):
            nodes = [p for p in members[b] if p < nn]
            cents = [p - nn for p in members[b] if p >= nn]
            dofs = list(nodes) + [nn + p for p in nodes]
            for k in cents:
                dofs += [2 * nn + 3 * k, 2 * nn + 3 * k + 1, 2 * nn + 3 * k + 2]
            self.leaf_dofs.append(np.array(dofs, dtype=np.int64))


# ----------------------------------------------------------------------------
# The factorisation
# ----------------------------------------------------------------------------

class IFMM:
    """IFMM factorisation of the completed double-layer matrix.

    ``order``: 'morton' eliminates the boxes of a level in Morton order;
    'color' eliminates them colour by colour ((ix mod 3, iy mod 3), Morton
    order inside a colour), the order a batched device implementation uses.
    """

    def __init__(self, geom, eps=1e-6, cheb_n=10, leaf_target=64, max_depth=0,
                 order="morton", dense=None):
        self.geom = geom
        self.eps = eps
        self.n = cheb_n
        self.tree = Tree(geom, leaf_target, max_depth)
        t = self.tree
        self.records = {}
        self._check_pores()
        a = dense if dense is not None else None
        lev = t.depth
        L = t.levels[lev]
        nn = geom.n_nodes
        wmask = dlp.wall_mask(geom)
        wall_len = geom.w[wmask].sum() if wmask.any() else 1.0
        self.wall_len = wall_len
        # ---- leaf-level operators (x = original unknowns of the box)
        S = {}
        dofs = t.leaf_dofs
        for b in range(len(L)):
            for c in L.neighbors[b]:
                if a is not None:
                    S[(b, c)] = a[np.ix_(dofs[b], dofs[c])]
                else:
                    S[(b, c)] = dlp.block(geom, dofs[b], dofs[c])
        n = cheb_n
        n2 = n * n
        phi, psi, gvec, hvec = [], [], [], []
        for b in range(len(L)):
            cx, cy = L.center[b]
            d = dofs[b]
            m = d.shape[0]
            ph = np.zeros((m, 2 * n2))
            ps = np.zeros((m, NSRC * n2))
            gv = np.zeros(m)
            hv = np.zeros(m)
            for r, dof in enumerate(d):
                if dof < 2 * nn:
                    i = dof if dof < nn else dof - nn
                    comp = 0 if dof < nn else 1
                    si = cheb_interp_2d(n, [geom.x[i]], [geom.y[i]], cx, cy, L.h)[0]
                    ph[r, comp * n2:(comp + 1) * n2] = si
                    nk = (geom.nx[i], geom.ny[i])
                    for kk in range(2):
                        col = 2 * kk + comp
                        ps[r, col * n2:(col + 1) * n2] = si * geom.w[i] * nk[kk]
                    if wmask[i]:
                        gv[r] = nk[comp]
                        hv[r] = geom.w[i] * nk[comp]
                else:
                    q = dof - 2 * nn
                    k, comp = q // 3, q % 3
                    sc = cheb_interp_2d(n, [geom.cx[k]], [geom.cy[k]], cx, cy, L.h)[0]
                    if comp < 2:
                        ps[r, (4 + comp) * n2:(5 + comp) * n2] = sc
                    else:
                        ps[r, 6 * n2:7 * n2] = sc * geom.radius[k]
            phi.append(ph)
            psi.append(ps)
            gvec.append(gv)
            hvec.append(hv)
        self.leaf_dofs = dofs
        self.levels_state = []
        rhs_dim = [d.shape[0] for d in dofs]
        while lev > t.root:
            L = t.levels[lev]
            uk, vk = kernel_bases(n, L.h, eps)
            W = []
            for b in range(len(L)):
                cols = [phi[b] @ uk, psi[b] @ vk]
                if np.any(gvec[b] != 0):
                    cols += [gvec[b][:, None], hvec[b][:, None]]
                W.append(orth_trunc(np.concatenate(cols, axis=1), eps))
            # initial couplings: Chebyshev M2L plus the rank-one wall term
            T = {}
            G = [W[b].T @ phi[b] for b in range(len(L))]
            H = [W[b].T @ psi[b] for b in range(len(L))]
            g0 = [W[b].T @ gvec[b] for b in range(len(L))]
            h0 = [W[b].T @ hvec[b] for b in range(len(L))]
            for b in range(len(L)):
                tx, ty = grid_points(n, *L.center[b], L.h)
                for c in L.ilist[b]:
                    sx, sy = grid_points(n, *L.center[c], L.h)
                    k = far_kernel(tx, ty, sx, sy)
                    T[(b, c)] = G[b] @ k @ H[c].T + np.outer(g0[b], h0[c]) / wall_len
            recs = self._eliminate_level(L, S, W, T, order)
            self.records[lev] = recs
            # ---- level change: build the parent system
            P = t.levels[lev - 1]
            r = [W[b].shape[1] for b in range(len(L))]
            off = {}
            pdim = []
            for p in range(len(P)):
                o = 0
                for c in P.children[p]:
                    off[c] = (p, o)
                    o += r[c]
                pdim.append(o)
            Sp = {}
            for p in range(len(P)):
                for q in P.neighbors[p]:
                    blk = np.zeros((pdim[p], pdim[q]))
                    for c in P.children[p]:
                        for d in P.children[q]:
                            tcd = T.get((c, d))
                            if tcd is not None:
                                _, oc = off[c]
                                _, od = off[d]
                                blk[oc:oc + r[c], od:od + r[d]] = _pad(tcd, r[c], r[d])
                    Sp[(p, q)] = blk
            nphi, npsi, ng, nh = [], [], [], []
            for p in range(len(P)):
                rows_phi, rows_psi, rows_g, rows_h = [], [], [], []
                pcx, pcy = P.center[p]
                gx, gy = grid_points(n, pcx, pcy, P.h)
                for c in P.children[p]:
                    ccx, ccy = L.center[c]
                    cgx, cgy = grid_points(n, ccx, ccy, L.h)
                    # parent Lagrange basis at the child's Chebyshev nodes
                    s_cp = cheb_interp_2d(n, cgx, cgy, pcx, pcy, P.h)
                    rows_phi.append((W[c].T @ phi[c]) @ np.kron(np.eye(2), s_cp))
                    rows_psi.append((W[c].T @ psi[c]) @ np.kron(np.eye(NSRC), s_cp))
                    rows_g.append(W[c].T @ gvec[c])
                    rows_h.append(W[c].T @ hvec[c])
                nphi.append(np.concatenate(rows_phi, axis=0))
                npsi.append(np.concatenate(rows_psi, axis=0))
                ng.append(np.concatenate(rows_g))
                nh.append(np.concatenate(rows_h))
            self.levels_state.append(dict(level=lev, offsets=off, ranks=r, pdim=pdim))
            phi, psi, gvec, hvec, S = nphi, npsi, ng, nh, Sp
            lev -= 1
        # ---- root: dense solve of what remains
        L = t.levels[lev]
        self.root_level = lev
        dims = [S[(b, b)].shape[0] for b in range(len(L))]
        offs = np.concatenate([[0], np.cumsum(dims)]).astype(int)
        big = np.zeros((offs[-1], offs[-1]))
        for b in range(len(L)):
            for c in L.neighbors[b]:
                big[offs[b]:offs[b + 1], offs[c]:offs[c + 1]] = S[(b, c)]
        self.root_offs = offs
        self.root_lu = sla.lu_factor(big) if offs[-1] else None
        self.max_rank = max([max(s["ranks"]) for s in self.levels_state] + [0])

    def _check_pores(self):
        g = self.geom
        h = self.tree.levels[self.tree.depth].h
        if g.n_pores and g.radius.max() >= h:
            raise ValueError("pore radius exceeds the leaf box side: constraint rows "
                             "would leave the near field")

    def _eliminate_level(self, L, S, W, T, order):
        eps = self.eps
        nb = len(L)
        if order == "color":
            seq = sorted(range(nb), key=lambda b: ((L.keys[b][0] % 3) * 3 + L.keys[b][1] % 3, b))
        else:
            seq = list(range(nb))
        gone = [False] * nb
        nset = [set(L.neighbors[b]) for b in range(nb)]
        recs = []
        for i in seq:
            act = [k for k in L.neighbors[i] if k != i and not gone[k]]
            sii = S[(i, i)]
            wi = W[i]
            lu = sla.lu_factor(sii)
            x = sla.lu_solve(lu, wi)
            y = sla.lu_solve(lu, wi, trans=1)
            piv = wi.T @ x
            pinv = np.linalg.inv(piv) if piv.shape[0] else piv
            sinv = sla.lu_solve(lu, np.eye(sii.shape[0]))
            axx = sinv - x @ pinv @ y.T
            axy = x @ pinv
            azx = pinv @ y.T
            s_ik = [S[(i, k)] for k in act]
            s_ki = [S[(k, i)] for k in act]
            recs.append(dict(i=i, act=act, s_ik=s_ik, s_ki=s_ki, axx=axx, axy=axy, azx=azx))
            # Schur complement: fill-ins among the active neighbours
            axx_sik = [axx @ sk for sk in s_ik]
            far = {}
            for jj, j in enumerate(act):
                for kk, k in enumerate(act):
                    f = -s_ki[jj] @ axx_sik[kk]
                    if k in nset[j]:
                        S[(j, k)] = S[(j, k)] + f
                    else:
                        far[(j, k)] = f
            bj = {j: s_ki[jj] @ axy for jj, j in enumerate(act)}      # R_j <- y_i
            gk = {k: azx @ s_ik[kk] for kk, k in enumerate(act)}      # Z_i <- x_k
            # recompression: augment the bases so that every fill-in that
            # must be redirected lies in their span (to tolerance eps)
            for j in act:
                cands = []
                if bj[j].shape[1]:
                    cands.append(bj[j])
                if gk[j].shape[0]:
                    cands.append(gk[j].T)
                for (a, b), f in far.items():
                    if a == j:
                        cands.append(f)
                    if b == j:
                        cands.append(f.T)
                W[j] = _augment(W[j], cands, eps)
            # couplings of the coarse system
            T[(i, i)] = _pad(T.get((i, i)), wi.shape[1], wi.shape[1]) + pinv
            for j in act:
                rj, ri = W[j].shape[1], wi.shape[1]
                T[(j, i)] = _pad(T.get((j, i)), rj, ri) + W[j].T @ bj[j]
                T[(i, j)] = _pad(T.get((i, j)), ri, rj) + gk[j] @ W[j]
            for (j, k), f in far.items():
                T[(j, k)] = _pad(T.get((j, k)), W[j].shape[1], W[k].shape[1]) + W[j].T @ f @ W[k]
            gone[i] = True
            for k in act:
                S.pop((i, k), None)
                S.pop((k, i), None)
            S.pop((i, i), None)
        return recs

    # ------------------------------------------------------------------------
    def solve(self, b: np.ndarray) -> np.ndarray:
        """x ~ A^{-1} b: forward substitution through the recorded
        eliminations (leaves to root), dense root solve, back substitution."""
        t = self.tree
        rhs = [b[d].copy() for d in self.leaf_dofs]
        saved = {}
        lev = t.depth
        for st in self.levels_state:
            recs = self.records[st["level"]]
            rz = {}
            gs = {}
            for rec in recs:
                i = rec["i"]
                g = rhs[i]
                gs[i] = g.copy()
                tt = rec["axx"] @ g
                for j, s_ji in zip(rec["act"], rec["s_ki"]):
                    rhs[j] = rhs[j] - s_ji @ tt
                rz[i] = rec["azx"] @ g
            saved[st["level"]] = gs
            P = t.levels[st["level"] - 1]
            new = []
            for p in range(len(P)):
                parts = [rz[c] for c in P.children[p]]
                new.append(np.concatenate(parts) if parts else np.zeros(0))
            rhs = new
        offs = self.root_offs
        full = np.concatenate(rhs) if rhs else np.zeros(0)
        xr = sla.lu_solve(self.root_lu, full) if offs[-1] else full
        x = [xr[offs[k]:offs[k + 1]] for k in range(len(offs) - 1)]
        for st in reversed(self.levels_state):
            lev = st["level"]
            L = t.levels[lev]
            y = [None] * len(L)
            for c, (p, o) in st["offsets"].items():
                y[c] = x[p][o:o + st["ranks"][c]]
            xs = [None] * len(L)
            gs = saved[lev]
            for rec in reversed(self.records[lev]):
                i = rec["i"]
                g = gs[i].copy()
                for k, s_ik in zip(rec["act"], rec["s_ik"]):
                    g -= s_ik @ xs[k]
                xs[i] = rec["axx"] @ g + rec["axy"] @ y[i]
            x = xs
        out = np.zeros_like(b)
        for d, v in zip(self.leaf_dofs, x):
            out[d] = v
        return out

    __call__ = solve


def _pad(m, r, c):
    if m is None:
        return np.zeros((r, c))
    if m.shape == (r, c):
        return m
    out = np.zeros((r, c))
    out[:m.shape[0], :m.shape[1]] = m
    return out


def _augment(w: np.ndarray, cands, eps: float) -> np.ndarray:
    """Recompression: W_new = [W, Q] where Q spans the part of the
    candidates outside span(W); each candidate block is first scaled by its
    Frobenius norm (relative eps; the norm is the reading recorded for the
    relative truncation of Section 3.3, the same on the GPU), then directions
    with singular value <= eps are dropped."""
    if not cands:
        return w
    parts = []
    for c in cands:
        if c.size == 0:
            continue
        s0 = np.linalg.norm(c)
        if s0 == 0:
            continue
        parts.append(c / s0)
    if not parts:
        return w
    c = np.concatenate(parts, axis=1)
    r = c - w @ (w.T @ c)
    r = r - w @ (w.T @ r)
    u, s, _ = np.linalg.svd(r, full_matrices=False)
    q = u[:, s > eps]
    if q.shape[1] == 0:
        return w
    q = q - w @ (w.T @ q)
    q, _ = np.linalg.qr(q)
    return np.concatenate([w, q], axis=1)
