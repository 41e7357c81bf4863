"""Space-time domain decomposition maps (integer data only).

Test infrastructure only (see the package docstring).

Follows Def. domdecom (overlapping boxes whose union covers Delta x Omega),
the local sizes nloc = n/p + 2 o (eqs. Eq-r, nlocx) and the closed local
intervals Delta_j = [t_j, t_{j+s_j}] (Sec. 3.2).  Readings:

* spatial pieces are given by latitude-band edges and, per band, longitude
  piece edges; a core is [band rows) x [piece cols); the extended box grows the
  core by ``o`` cells on every side, clipped at the poles and wrapped in
  longitude; a band with a single piece gives a box spanning the whole circle;
* time intervals [T_j, T_{j+1}] grow by ``o_t`` levels on each side, clipped to
  [0, N_t], and are closed: levels S_j .. E_j;
* subdomain index s = j * (number of spatial pieces) + i, pieces band-major;
* halo ring (lateral boundary of the restricted model, eq. restricted): every
  neighbour position just outside the box that the 5-point stencil reads.
  Positions are numbered south row (box row -1, cols 0..nx-1), north row (box
  row ny), west column (box col -1, rows 0..ny-1), east column (box col nx).
  A position is *internal* when the box spans all longitudes and the position
  lies across the east/west seam or across a pole; it then reads the box
  itself.  Otherwise it is frozen and reads the core owner of the (pole-mapped)
  cell in the same time interval; u and v change sign across a pole;
* under the Turkel-Zwas variant (offsets p, q) the stencil reads up to q rows
  and p columns beyond the box, corners included, so the ring becomes a pad:
  for a box of several pieces every position of the frame [-q, ny+q) x
  [-p, nx+p) outside the box, numbered south block (rows -q..-1, columns
  -p..nx+p-1, row-major), north block (rows ny..ny+q-1), west block (rows
  0..ny-1, columns -p..-1), east block (columns nx..nx+p-1); for a box
  spanning the circle only the south and north blocks over columns 0..nx-1
  (its columns wrap onto itself).  A row beyond a pole maps to the row at
  the same depth on the other side, half a circle further, u and v negated.
  A position of a spanning box that maps into the box itself is internal;
  every other position is frozen and reads the core owner of the mapped cell
  in the same time interval;
* restriction weights (Def. defrestrfun, applied to squared terms):
  c(n, cell) = number of extended space-time boxes containing (n, cell), which
  is the spatial count times the temporal count;
* overlap neighbours (eqs. overl, ospatial, otime): every other subdomain
  whose extended space-time box intersects, diagonal ones included.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Box:
    sub: int
    piece: int
    interval: int
    band: int
    core_row0: int
    core_row1: int
    core_col0: int
    core_col1: int
    row0: int
    ny: int
    col0: int
    nx: int
    span: bool
    lev0: int          # S_j
    nlev: int          # E_j - S_j + 1
    pad_p: int = 0     # Turkel-Zwas pad widths (0: the one-cell ring)
    pad_q: int = 0

    @property
    def ncell(self):
        return self.ny * self.nx

    @property
    def nring(self):
        p, q = self.pad_p, self.pad_q
        if q == 0:
            return 2 * self.nx + 2 * self.ny
        if self.span:
            return 2 * q * self.nx
        return 2 * q * (self.nx + 2 * p) + 2 * p * self.ny


def ring_coords(b: Box):
    """Box-relative (row, col) of every ring (or pad) position, in order."""
    ny, nx, p, q = b.ny, b.nx, b.pad_p, b.pad_q
    if q == 0:
        rr = np.concatenate([np.full(nx, -1), np.full(nx, ny), np.arange(ny), np.arange(ny)])
        cc = np.concatenate([np.arange(nx), np.arange(nx), np.full(ny, -1), np.full(ny, nx)])
        return rr, cc
    cols = np.arange(nx) if b.span else np.arange(-p, nx + p)
    south = np.arange(-q, 0)
    north = np.arange(ny, ny + q)
    rr = [np.repeat(south, cols.size), np.repeat(north, cols.size)]
    cc = [np.tile(cols, q), np.tile(cols, q)]
    if not b.span:
        rr += [np.repeat(np.arange(ny), p), np.repeat(np.arange(ny), p)]
        cc += [np.tile(np.arange(-p, 0), ny), np.tile(np.arange(nx, nx + p), ny)]
    return np.concatenate(rr), np.concatenate(cc)


@dataclasses.dataclass
class DDMaps:
    nlat: int
    nlon: int
    nsteps: int
    nspace: int
    ntime: int
    boxes: list
    owner: np.ndarray          # [nlat][nlon] piece owning each core cell
    cover_sp: np.ndarray       # [nlat][nlon] number of extended spatial boxes
    time_count: np.ndarray     # [nsteps+1] number of extended intervals
    halo_src: list             # per s: int32 [nring], source subdomain or -1
    halo_off: list             # per s: int32 [nring], cell offset in source box
    halo_sign: list            # per s: int32 [nring], +1 / -1 (u, v only)
    neighbors: list            # per s: int32 sorted neighbour subdomains
    obs_bin: list              # per s: int64 sorted global observation indices

    def box_cells_global(self, b: Box):
        """Global (row, col) of every box cell, row-major in the box."""
        rows = b.row0 + np.arange(b.ny)
        cols = (b.col0 + np.arange(b.nx)) % self.nlon
        return np.repeat(rows, b.nx), np.tile(cols, b.ny)

    def box_index(self, b: Box, grow, gcol):
        """Box cell index of global cells, -1 where outside the box."""
        r = np.asarray(grow) - b.row0
        c = (np.asarray(gcol) - b.col0) % self.nlon
        ok = (r >= 0) & (r < b.ny) & (c < b.nx)
        return np.where(ok, r * b.nx + c, -1)


def _pieces(prob):
    edges = np.asarray(prob.band_lat_edges, dtype=np.int64)
    npc = np.asarray(prob.band_npieces, dtype=np.int64)
    lon = np.asarray(prob.piece_lon_edges, dtype=np.int64)
    out = []
    pos = 0
    for b in range(len(npc)):
        le = lon[pos:pos + npc[b] + 1]
        pos += npc[b] + 1
        for p in range(npc[b]):
            out.append((b, int(edges[b]), int(edges[b + 1]), int(le[p]), int(le[p + 1]),
                        int(npc[b])))
    return out


def build(prob) -> DDMaps:
    nlat, nlon, nt = prob.nlat, prob.nlon, prob.nsteps
    o, ot = prob.overlap_cells, prob.overlap_steps
    pieces = _pieces(prob)
    nspace = len(pieces)
    tzp = int(getattr(prob, "tz_p", 0))
    pp, pq = (tzp, int(prob.tz_q)) if tzp > 0 else (0, 0)
    tedges = np.asarray(prob.time_edges, dtype=np.int64)
    ntime = len(tedges) - 1

    boxes = []
    for j in range(ntime):
        S = max(0, int(tedges[j]) - ot)
        E = min(nt, int(tedges[j + 1]) + ot)
        for i, (b, r0, r1, c0, c1, npc) in enumerate(pieces):
            br0 = max(0, r0 - o)
            br1 = min(nlat, r1 + o)
            if npc == 1:
                col0, nx, span = 0, nlon, True
            else:
                col0, nx, span = (c0 - o) % nlon, (c1 - c0) + 2 * o, False
                if nx + 2 * pp > nlon:
                    raise ValueError("a box and its pad columns must not wrap the circle")
            boxes.append(Box(sub=j * nspace + i, piece=i, interval=j, band=b,
                             core_row0=r0, core_row1=r1, core_col0=c0, core_col1=c1,
                             row0=br0, ny=br1 - br0, col0=col0, nx=nx, span=span,
                             lev0=S, nlev=E - S + 1, pad_p=pp, pad_q=pq))

    owner = np.full((nlat, nlon), -1, dtype=np.int64)
    for i, (b, r0, r1, c0, c1, npc) in enumerate(pieces):
        owner[r0:r1, c0:c1] = i
    assert (owner >= 0).all(), "cores do not tile the grid"

    cover_sp = np.zeros((nlat, nlon), dtype=np.int64)
    for bx in boxes[:nspace]:
        cols = (bx.col0 + np.arange(bx.nx)) % nlon
        cover_sp[bx.row0:bx.row0 + bx.ny][:, cols] += 1

    time_count = np.zeros(nt + 1, dtype=np.int64)
    for j in range(ntime):
        bx = boxes[j * nspace]
        time_count[bx.lev0:bx.lev0 + bx.nlev] += 1

    half = nlon // 2
    halo_src, halo_off, halo_sign = [], [], []
    for bx in boxes:
        ny, nx = bx.ny, bx.nx
        # box-relative (row, col) of each ring position
        rr, cc = ring_coords(bx)
        src = np.empty(rr.size, dtype=np.int64)
        off = np.empty(rr.size, dtype=np.int64)
        sgn = np.ones(rr.size, dtype=np.int64)
        for k in range(rr.size):
            r, c = int(rr[k]), int(cc[k])
            grow = bx.row0 + r
            across = grow < 0 or grow >= nlat
            if bx.span and (c < 0 or c >= nx):
                src[k], off[k] = -1, r * nx + (c % nx)
                continue
            # the row at the same depth beyond the pole, half a circle further
            mrow = -1 - grow if grow < 0 else (2 * nlat - 1 - grow if grow >= nlat else grow)
            if bx.span and across and bx.row0 <= mrow < bx.row0 + ny:
                src[k], off[k], sgn[k] = -1, (mrow - bx.row0) * nx + (c + half) % nx, -1
                continue
            gcol = (bx.col0 + c) % nlon
            if across:
                mcol = (gcol + half) % nlon
                sgn[k] = -1
            else:
                mcol = gcol
            sb = boxes[bx.interval * nspace + owner[mrow, mcol]]
            src[k] = sb.sub
            rel_r = mrow - sb.row0
            rel_c = (mcol - sb.col0) % nlon
            assert 0 <= rel_r < sb.ny and rel_c < sb.nx
            off[k] = rel_r * sb.nx + rel_c
        halo_src.append(src.astype(np.int32))
        halo_off.append(off.astype(np.int32))
        halo_sign.append(sgn.astype(np.int32))

    def spatial_meet(a: Box, b: Box):
        if a.row0 >= b.row0 + b.ny or b.row0 >= a.row0 + a.ny:
            return False
        if a.span or b.span:
            return True
        return ((b.col0 - a.col0) % nlon < a.nx) or ((a.col0 - b.col0) % nlon < b.nx)

    # boxes of one interval share the spatial pieces, so the spatial test is
    # done once per pair of pieces and the temporal one once per pair of
    # intervals
    smeet = [[i2 for i2 in range(nspace) if spatial_meet(boxes[i], boxes[i2])]
             for i in range(nspace)]
    tmeet = []
    for j in range(ntime):
        a = boxes[j * nspace]
        tmeet.append([j2 for j2 in range(ntime)
                      if not (a.lev0 > boxes[j2 * nspace].lev0 + boxes[j2 * nspace].nlev - 1
                              or boxes[j2 * nspace].lev0 > a.lev0 + a.nlev - 1)])
    neighbors = []
    for a in boxes:
        nb = [j2 * nspace + i2 for j2 in tmeet[a.interval] for i2 in smeet[a.piece]
              if j2 * nspace + i2 != a.sub]
        neighbors.append(np.array(sorted(nb), dtype=np.int32))

    # observation bins: candidates by level range (observations sorted by
    # step), then the in-box test
    ostep = np.asarray(prob.obs_step, dtype=np.int64)
    ocell = np.asarray(prob.obs_cell, dtype=np.int64)
    order = np.argsort(ostep, kind="stable")
    ssorted = ostep[order]
    obs_bin = []
    for bx in boxes:
        lo = np.searchsorted(ssorted, bx.lev0, side="left")
        hi = np.searchsorted(ssorted, bx.lev0 + bx.nlev - 1, side="right")
        cand = order[lo:hi]
        r = ocell[cand] // nlon - bx.row0
        c = (ocell[cand] % nlon - bx.col0) % nlon
        inbox = (r >= 0) & (r < bx.ny) & (c < bx.nx)
        obs_bin.append(np.sort(cand[inbox]).astype(np.int64))

    return DDMaps(nlat=nlat, nlon=nlon, nsteps=nt, nspace=nspace, ntime=ntime,
                  boxes=boxes, owner=owner, cover_sp=cover_sp, time_count=time_count,
                  halo_src=halo_src, halo_off=halo_off, halo_sign=halo_sign,
                  neighbors=neighbors, obs_bin=obs_bin)
