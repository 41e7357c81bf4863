// Host-side construction of the space-time decomposition maps.
//
// Boxes (Def. domdecom; local sizes n/p + 2o of eqs. Eq-r, nlocx): a core is
// [band rows) x [piece cols); its extended box grows by o cells per side,
// clipped at the poles and wrapped in longitude; a band with one piece gives
// a box spanning the circle.  Intervals [T_j, T_{j+1}] grow by o_t levels
// per side, clipped to [0, N_t], closed (Sec. 3.2).  Subdomain index
// s = j * nspace + i with pieces numbered band-major.
//
// Halo ring = lateral boundary of the restricted model (eq. restricted): the
// positions just outside the box read by the 5-point stencil, numbered south
// row, north row, west column, east column.  A position wraps inside the box
// (source -1) when the box spans the circle and the position is across the
// seam or across a pole; otherwise it is frozen and read from the core owner
// of the pole-mapped cell in the same interval, with u, v negated across a
// pole.
//
// Restriction weights (Def. defrestrfun applied to squared terms): counts of
// extended boxes covering a point; the space-time count is the spatial count
// times the interval count because every interval uses the same spatial
// pieces.  Overlap neighbours (eqs. overl, ospatial, otime): every other
// subdomain whose extended space-time box intersects.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <sstream>
#include <unordered_set>

namespace dd4dvar {

namespace {
thread_local std::string g_thread_error;

struct Invalid {
  std::string msg;
};

void require(bool ok, const std::string& msg) {
  if (!ok) throw Invalid{msg};
}

int64_t mod(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

// Box-relative (row, col) of ring position k.  One-cell ring: south row,
// north row, west column, east column.  Turkel-Zwas pad (offsets p, q): the
// south block (rows -q..-1) and the north block (rows ny..ny+q-1), row-major
// over columns -p..nx+p-1 (0..nx-1 for a box spanning the circle), then for
// a box of several pieces the west block (rows 0..ny-1, columns -p..-1) and
// the east block (columns nx..nx+p-1), row-major.
void ring_coord(const BoxInfo& b, int k, int* r, int* c) {
  const int ny = b.ny, nx = b.nx, p = b.pad_p, q = b.pad_q;
  if (q == 0) {
    if (k < nx) { *r = -1; *c = k; }
    else if (k < 2 * nx) { *r = ny; *c = k - nx; }
    else if (k < 2 * nx + ny) { *r = k - 2 * nx; *c = -1; }
    else { *r = k - 2 * nx - ny; *c = nx; }
    return;
  }
  const int w = b.span ? nx : nx + 2 * p, c0 = b.span ? 0 : -p;
  if (k < 2 * q * w) {
    const int row = k / w;
    *r = row < q ? row - q : ny + (row - q);
    *c = c0 + k % w;
    return;
  }
  k -= 2 * q * w;
  const int east = k >= ny * p;
  if (east) k -= ny * p;
  *r = k / p;
  *c = east ? nx + k % p : -p + k % p;
}
}  // namespace

void set_thread_error(const std::string& msg) { g_thread_error = msg; }
const char* thread_error() { return g_thread_error.c_str(); }

static void validate_and_copy(const dd4dvar_model_desc* m,
                              const dd4dvar_partition_desc* p,
                              const dd4dvar_data_desc* d, dd4dvar_plan* plan) {
  require(m && p && d, "null descriptor");
  require(m->nlat >= 2, "nlat must be >= 2");
  require(m->nlon >= 4 && m->nlon % 2 == 0, "nlon must be even and >= 4");
  require(m->nsteps >= 1, "nsteps must be >= 1");
  require(int64_t(m->nlat) * m->nlon <= (int64_t(1) << 30), "grid too large");
  require(std::isfinite(m->dt) && m->dt > 0, "dt must be > 0");
  require(std::isfinite(m->radius) && m->radius > 0, "radius must be > 0");
  require(std::isfinite(m->gravity) && m->gravity > 0, "gravity must be > 0");
  require(std::isfinite(m->omega), "omega must be finite");
  require(std::isfinite(m->h_ref), "h_ref must be finite");
  require(std::isfinite(m->lambda_obs) && m->lambda_obs >= 0, "lambda_obs must be >= 0");
  require(std::isfinite(m->mu_overlap) && m->mu_overlap >= 0, "mu_overlap must be >= 0");
  require(m->precision == DD4DVAR_FP64 || m->precision == DD4DVAR_FP32_STATE,
          "unknown precision");
  require(m->weight_mode == 0 || m->weight_mode == 1, "unknown weight_mode");
  if (m->tz_p != 0) {
    require(m->tz_p >= 1 && m->tz_p <= m->nlon / 2, "tz_p must be 0 or in 1..nlon/2");
    require(m->tz_q >= 1 && m->tz_q <= m->nlat / 2, "tz_q must be in 1..nlat/2");
    require(std::isfinite(m->tz_alpha) && m->tz_alpha >= 0 && m->tz_alpha <= 1,
            "tz_alpha must be in [0, 1]");
  }
  plan->model = *m;

  const int nlat = m->nlat, nlon = m->nlon, nt = m->nsteps;
  require(p->n_bands >= 1 && p->band_lat_edges && p->band_npieces && p->piece_lon_edges,
          "partition arrays missing");
  require(p->band_lat_edges[0] == 0 && p->band_lat_edges[p->n_bands] == nlat,
          "band edges must run 0..nlat");
  for (int b = 0; b < p->n_bands; ++b)
    require(p->band_lat_edges[b + 1] > p->band_lat_edges[b], "band edges must increase");
  require(p->n_time >= 1 && p->time_edges, "time edges missing");
  require(p->time_edges[0] == 0 && p->time_edges[p->n_time] == nt,
          "time edges must run 0..nsteps");
  for (int j = 0; j < p->n_time; ++j)
    require(p->time_edges[j + 1] > p->time_edges[j], "time edges must increase");
  const int o = p->overlap_cells, ot = p->overlap_steps;
  require(o >= 0 && ot >= 0, "overlaps must be >= 0");
  for (int j = 0; j < p->n_time; ++j)
    require(p->time_edges[j + 1] - p->time_edges[j] >= ot,
            "overlap_steps exceeds an interval length");
  int64_t pos = 0;
  for (int b = 0; b < p->n_bands; ++b) {
    const int np = p->band_npieces[b];
    require(np >= 1, "band_npieces must be >= 1");
    const int32_t* le = p->piece_lon_edges + pos;
    require(le[0] == 0 && le[np] == nlon, "piece edges must run 0..nlon");
    require(p->band_lat_edges[b + 1] - p->band_lat_edges[b] >= o,
            "overlap_cells exceeds a band height");
    for (int q = 0; q < np; ++q) {
      require(le[q + 1] > le[q], "piece edges must increase");
      if (np > 1) {
        require(le[q + 1] - le[q] >= o, "overlap_cells exceeds a piece width");
        require(le[q + 1] - le[q] + 2 * o < nlon, "extended piece wraps onto itself");
      }
    }
    pos += np + 1;
  }

  const int64_t ncell = int64_t(nlat) * nlon;
  require(d->xb0 && d->sigma_b, "background arrays missing");
  plan->xb0.assign(d->xb0, d->xb0 + 3 * ncell);
  for (double v : plan->xb0) require(std::isfinite(v), "xb0 must be finite");
  plan->sigma_b.assign(d->sigma_b, d->sigma_b + 3);
  for (double v : plan->sigma_b) require(std::isfinite(v) && v > 0, "sigma_b must be > 0");
  require(d->nobs >= 0 && d->nobs < (int64_t(1) << 31), "bad nobs");
  const int64_t nobs = d->nobs;
  if (nobs > 0)
    require(d->obs_step && d->obs_cell && d->obs_field && d->obs_value && d->obs_sigma,
            "observation arrays missing");
  plan->obs_step.assign(d->obs_step, d->obs_step + nobs);
  plan->obs_cell.assign(d->obs_cell, d->obs_cell + nobs);
  plan->obs_field.assign(d->obs_field, d->obs_field + nobs);
  plan->obs_value.assign(d->obs_value, d->obs_value + nobs);
  plan->obs_sigma.assign(d->obs_sigma, d->obs_sigma + nobs);
  std::vector<uint64_t> keys(nobs);
  for (int64_t k = 0; k < nobs; ++k) {
    const int32_t st = plan->obs_step[k], c = plan->obs_cell[k], f = plan->obs_field[k];
    require(st >= 0 && st <= nt, "observation step out of range");
    require(c >= 0 && c < ncell, "observation cell out of range");
    require(f >= 0 && f <= 2, "observation field out of range");
    require(std::isfinite(plan->obs_value[k]), "observation value not finite");
    require(std::isfinite(plan->obs_sigma[k]) && plan->obs_sigma[k] > 0,
            "observation sigma must be > 0");
    keys[k] = (uint64_t(st) * uint64_t(ncell) + uint64_t(c)) * 4u + uint64_t(f);
  }
  std::sort(keys.begin(), keys.end());
  require(std::adjacent_find(keys.begin(), keys.end()) == keys.end(),
          "duplicate observation (step, cell, field)");
}

dd4dvar_status build_plan(const dd4dvar_model_desc* m, const dd4dvar_partition_desc* p,
                          const dd4dvar_data_desc* d, dd4dvar_plan* plan,
                          std::string* err) {
  try {
    validate_and_copy(m, p, d, plan);
    const int nlat = m->nlat, nlon = m->nlon, nt = m->nsteps;
    const int o = p->overlap_cells, ot = p->overlap_steps;
    const int64_t ncell = int64_t(nlat) * nlon;
    const int half = nlon / 2;

    // spatial pieces, band-major
    struct Piece { int band, r0, r1, c0, c1, np; };
    std::vector<Piece> pieces;
    int64_t pos = 0;
    for (int b = 0; b < p->n_bands; ++b) {
      const int np = p->band_npieces[b];
      for (int q = 0; q < np; ++q)
        pieces.push_back({b, p->band_lat_edges[b], p->band_lat_edges[b + 1],
                          p->piece_lon_edges[pos + q], p->piece_lon_edges[pos + q + 1], np});
      pos += np + 1;
    }
    const int nspace = int(pieces.size());
    const int ntime = p->n_time;
    plan->nspace = nspace;
    plan->ntime = ntime;
    plan->nsub = nspace * ntime;

    plan->owner.assign(ncell, -1);
    for (int i = 0; i < nspace; ++i)
      for (int r = pieces[i].r0; r < pieces[i].r1; ++r)
        for (int c = pieces[i].c0; c < pieces[i].c1; ++c) plan->owner[int64_t(r) * nlon + c] = i;

    plan->boxes.clear();
    int64_t ctrl = 0, traj = 0;
    for (int j = 0; j < ntime; ++j) {
      const int S = std::max(0, p->time_edges[j] - ot);
      const int E = std::min(nt, p->time_edges[j + 1] + ot);
      for (int i = 0; i < nspace; ++i) {
        const Piece& pc = pieces[i];
        BoxInfo bx{};
        bx.sub = j * nspace + i;
        bx.piece = i;
        bx.interval = j;
        bx.band = pc.band;
        bx.core_r0 = pc.r0; bx.core_r1 = pc.r1; bx.core_c0 = pc.c0; bx.core_c1 = pc.c1;
        bx.row0 = std::max(0, pc.r0 - o);
        bx.ny = std::min(nlat, pc.r1 + o) - bx.row0;
        if (pc.np == 1) {
          bx.col0 = 0; bx.nx = nlon; bx.span = 1;
        } else {
          bx.col0 = int(mod(pc.c0 - o, nlon)); bx.nx = pc.c1 - pc.c0 + 2 * o; bx.span = 0;
          if (bx.nx + 2 * m->tz_p > nlon)
            throw Invalid{"a box and its Turkel-Zwas pad columns must not wrap the circle"};
        }
        bx.pole_s = bx.span && bx.row0 == 0;
        bx.pole_n = bx.span && bx.row0 + bx.ny == nlat;
        bx.lev0 = S;
        bx.nlev = E - S + 1;
        bx.pad_p = m->tz_p > 0 ? m->tz_p : 0;
        bx.pad_q = m->tz_p > 0 ? m->tz_q : 0;
        if (bx.pad_q == 0)
          bx.nring = 2 * bx.nx + 2 * bx.ny;
        else if (bx.span)
          bx.nring = 2 * bx.pad_q * bx.nx;
        else
          bx.nring = 2 * bx.pad_q * (bx.nx + 2 * bx.pad_p) + 2 * bx.pad_p * bx.ny;
        bx.ctrl_off = ctrl;
        bx.traj_off = traj;
        ctrl += 3 * bx.ncell();
        traj += int64_t(bx.nlev) * 3 * bx.ncell();
        plan->boxes.push_back(bx);
      }
    }
    plan->ctrl_total = ctrl;
    plan->traj_total = traj;

    // spatial coverage counts
    plan->cover_sp.assign(ncell, 0);
    for (int i = 0; i < nspace; ++i) {
      const BoxInfo& bx = plan->boxes[i];
      for (int r = 0; r < bx.ny; ++r)
        for (int c = 0; c < bx.nx; ++c)
          plan->cover_sp[int64_t(bx.row0 + r) * nlon + mod(bx.col0 + c, nlon)] += 1;
    }
    plan->time_count.assign(nt + 1, 0);
    for (int j = 0; j < ntime; ++j) {
      const BoxInfo& bx = plan->boxes[int64_t(j) * nspace];
      for (int n = bx.lev0; n < bx.lev0 + bx.nlev; ++n) plan->time_count[n] += 1;
    }
    plan->cell_ptr.assign(plan->nsub + 1, 0);
    for (int s = 0; s < plan->nsub; ++s)
      plan->cell_ptr[s + 1] = plan->cell_ptr[s] + plan->boxes[s].ncell();
    plan->cover_box.resize(plan->cell_ptr[plan->nsub]);
    for (int s = 0; s < plan->nsub; ++s) {
      const BoxInfo& bx = plan->boxes[s];
      int32_t* out = plan->cover_box.data() + plan->cell_ptr[s];
      for (int r = 0; r < bx.ny; ++r)
        for (int c = 0; c < bx.nx; ++c)
          out[int64_t(r) * bx.nx + c] =
              plan->cover_sp[int64_t(bx.row0 + r) * nlon + mod(bx.col0 + c, nlon)];
    }

    // halo rings
    plan->ring_ptr.assign(plan->nsub + 1, 0);
    for (int s = 0; s < plan->nsub; ++s)
      plan->ring_ptr[s + 1] = plan->ring_ptr[s] + plan->boxes[s].nring;
    const int64_t nr = plan->ring_ptr[plan->nsub];
    plan->halo_src.assign(nr, -1);
    plan->halo_off.assign(nr, 0);
    plan->halo_sign.assign(nr, 1);
    plan->halo_gcell.assign(nr, -1);
    for (int s = 0; s < plan->nsub; ++s) {
      const BoxInfo& bx = plan->boxes[s];
      const int64_t base = plan->ring_ptr[s];
      for (int k = 0; k < bx.nring; ++k) {
        int r, c;
        ring_coord(bx, k, &r, &c);
        const int grow = bx.row0 + r;
        const bool across = grow < 0 || grow >= nlat;
        if (bx.span && (c < 0 || c >= bx.nx)) {
          plan->halo_src[base + k] = -1;
          plan->halo_off[base + k] = r * bx.nx + int(mod(c, bx.nx));
          continue;
        }
        // the row at the same depth beyond the pole, half a circle further
        const int mrow = grow < 0 ? -1 - grow : (grow >= nlat ? 2 * nlat - 1 - grow : grow);
        if (bx.span && across && mrow >= bx.row0 && mrow < bx.row0 + bx.ny) {
          plan->halo_src[base + k] = -1;
          plan->halo_off[base + k] = (mrow - bx.row0) * bx.nx + int(mod(c + half, bx.nx));
          plan->halo_sign[base + k] = -1;
          continue;
        }
        const int gcol = int(mod(bx.col0 + c, nlon));
        int mcol = gcol;
        if (across) {
          mcol = int(mod(gcol + half, nlon));
          plan->halo_sign[base + k] = -1;
        }
        const int src = bx.interval * nspace + plan->owner[int64_t(mrow) * nlon + mcol];
        const BoxInfo& sb = plan->boxes[src];
        const int rr = mrow - sb.row0;
        const int cc = int(mod(mcol - sb.col0, nlon));
        if (rr < 0 || rr >= sb.ny || cc >= sb.nx) throw Invalid{"internal: ring source outside box"};
        plan->halo_src[base + k] = src;
        plan->halo_off[base + k] = rr * sb.nx + cc;
        plan->halo_gcell[base + k] = mrow * nlon + mcol;
      }
    }

    // overlap neighbours
    auto spatial_meet = [&](const BoxInfo& a, const BoxInfo& b) {
      if (a.row0 >= b.row0 + b.ny || b.row0 >= a.row0 + a.ny) return false;
      if (a.span || b.span) return true;
      return mod(b.col0 - a.col0, nlon) < a.nx || mod(a.col0 - b.col0, nlon) < b.nx;
    };
    std::vector<char> meet(size_t(nspace) * nspace, 0);
    for (int a = 0; a < nspace; ++a)
      for (int b = 0; b < nspace; ++b)
        meet[size_t(a) * nspace + b] = spatial_meet(plan->boxes[a], plan->boxes[b]);
    plan->nbr_ptr.assign(plan->nsub + 1, 0);
    plan->nbr_idx.clear();
    for (int s = 0; s < plan->nsub; ++s) {
      const BoxInfo& a = plan->boxes[s];
      for (int t = 0; t < plan->nsub; ++t) {
        if (t == s) continue;
        const BoxInfo& b = plan->boxes[t];
        if (a.lev0 > b.lev0 + b.nlev - 1 || b.lev0 > a.lev0 + a.nlev - 1) continue;
        if (meet[size_t(a.piece) * nspace + b.piece]) plan->nbr_idx.push_back(t);
      }
      plan->nbr_ptr[s + 1] = int64_t(plan->nbr_idx.size());
    }

    // observation bins: covering pieces per cell (CSR), then per observation
    std::vector<int64_t> cptr(ncell + 1, 0);
    for (int64_t c = 0; c < ncell; ++c) cptr[c + 1] = cptr[c] + plan->cover_sp[c];
    std::vector<int32_t> cpiece(cptr[ncell]);
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int i = 0; i < nspace; ++i) {
      const BoxInfo& bx = plan->boxes[i];
      for (int r = 0; r < bx.ny; ++r)
        for (int c = 0; c < bx.nx; ++c) {
          const int64_t g = int64_t(bx.row0 + r) * nlon + mod(bx.col0 + c, nlon);
          cpiece[fill[g]++] = i;
        }
    }
    std::vector<std::vector<int32_t>> bins(plan->nsub);
    const int64_t nobs = int64_t(plan->obs_step.size());
    for (int64_t k = 0; k < nobs; ++k) {
      const int st = plan->obs_step[k];
      const int64_t c = plan->obs_cell[k];
      for (int j = 0; j < ntime; ++j) {
        const BoxInfo& bj = plan->boxes[int64_t(j) * nspace];
        if (st < bj.lev0 || st > bj.lev0 + bj.nlev - 1) continue;
        for (int64_t q = cptr[c]; q < cptr[c + 1]; ++q)
          bins[int64_t(j) * nspace + cpiece[q]].push_back(int32_t(k));
      }
    }
    plan->obs_ptr.assign(plan->nsub + 1, 0);
    plan->obs_idx.clear();
    for (int s = 0; s < plan->nsub; ++s) {
      plan->obs_idx.insert(plan->obs_idx.end(), bins[s].begin(), bins[s].end());
      plan->obs_ptr[s + 1] = int64_t(plan->obs_idx.size());
    }
    return DD4DVAR_OK;
  } catch (const Invalid& e) {
    if (err) *err = e.msg;
    return DD4DVAR_E_INVALID;
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    return DD4DVAR_E_NOMEM;
  }
}

}  // namespace dd4dvar

using dd4dvar::BoxInfo;

extern "C" {

dd4dvar_status dd4dvar_plan_create(const dd4dvar_model_desc* model,
                                   const dd4dvar_partition_desc* part,
                                   const dd4dvar_data_desc* data, dd4dvar_plan** out) {
  if (!out) {
    dd4dvar::set_thread_error("null output pointer");
    return DD4DVAR_E_INVALID;
  }
  *out = nullptr;
  dd4dvar_plan* plan = new (std::nothrow) dd4dvar_plan();
  if (!plan) {
    dd4dvar::set_thread_error("host allocation failed");
    return DD4DVAR_E_NOMEM;
  }
  std::string err;
  dd4dvar_status st = dd4dvar::build_plan(model, part, data, plan, &err);
  if (st != DD4DVAR_OK) {
    dd4dvar::set_thread_error(err);
    delete plan;
    return st;
  }
  dd4dvar::set_thread_error("");
  *out = plan;
  return DD4DVAR_OK;
}

void dd4dvar_plan_destroy(dd4dvar_plan* plan) { delete plan; }

dd4dvar_status dd4dvar_plan_sizes(const dd4dvar_plan* plan, int32_t* nsub, int64_t* ctrl_len,
                                  int64_t* traj_len) {
  if (!plan) return DD4DVAR_E_INVALID;
  if (nsub) *nsub = plan->nsub;
  if (ctrl_len) *ctrl_len = plan->ctrl_total;
  if (traj_len) *traj_len = plan->traj_total;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_plan_subdomain_info(const dd4dvar_plan* plan, int32_t s, int64_t out[10]) {
  if (!plan || !out || s < 0 || s >= plan->nsub) return DD4DVAR_E_INVALID;
  const BoxInfo& b = plan->boxes[s];
  const int64_t v[10] = {b.row0, b.ny, b.col0, b.nx, b.lev0, b.nlev, b.ctrl_off, b.traj_off,
                         b.span, b.nring};
  std::memcpy(out, v, sizeof(v));
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_plan_get_map(const dd4dvar_plan* plan, int32_t kind, int32_t s,
                                    int64_t* len, int32_t* buf) {
  if (!plan || !len) return DD4DVAR_E_INVALID;
  const int32_t* src = nullptr;
  int64_t n = 0;
  if (kind == 4) {
    src = plan->time_count.data();
    n = int64_t(plan->time_count.size());
  } else {
    if (s < 0 || s >= plan->nsub) return DD4DVAR_E_INVALID;
    switch (kind) {
      case 0: case 1: case 2: case 7: {
        const std::vector<int32_t>& v = kind == 0 ? plan->halo_src
                                        : kind == 1 ? plan->halo_off
                                        : kind == 2 ? plan->halo_sign : plan->halo_gcell;
        src = v.data() + plan->ring_ptr[s];
        n = plan->ring_ptr[s + 1] - plan->ring_ptr[s];
        break;
      }
      case 3:
        src = plan->cover_box.data() + plan->cell_ptr[s];
        n = plan->cell_ptr[s + 1] - plan->cell_ptr[s];
        break;
      case 5:
        src = plan->nbr_idx.data() + plan->nbr_ptr[s];
        n = plan->nbr_ptr[s + 1] - plan->nbr_ptr[s];
        break;
      case 6:
        src = plan->obs_idx.data() + plan->obs_ptr[s];
        n = plan->obs_ptr[s + 1] - plan->obs_ptr[s];
        break;
      default:
        return DD4DVAR_E_INVALID;
    }
  }
  if (!buf) {
    *len = n;
    return DD4DVAR_OK;
  }
  if (*len < n) return DD4DVAR_E_INVALID;
  if (n) std::memcpy(buf, src, size_t(n) * sizeof(int32_t));
  *len = n;
  return DD4DVAR_OK;
}

}  // extern "C"
