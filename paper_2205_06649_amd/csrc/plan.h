// Host-side plan of the space-time decomposition: boxes, halo maps, counts,
// overlap neighbours and observation bins (Def. domdecom, eqs. Eq-r, nlocx,
// Def. defrestrfun, eqs. overl/ospatial/otime).  Pure C++, no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dd4dvar.h"

namespace dd4dvar {

struct BoxInfo {
  int32_t sub, piece, interval, band;
  int32_t core_r0, core_r1, core_c0, core_c1;
  int32_t row0, ny, col0, nx;
  int32_t span;          // box covers every longitude (band of one piece)
  int32_t pole_s, pole_n;  // span box touching the south / north pole row
  int32_t lev0, nlev;    // levels S_j .. S_j + nlev - 1
  int32_t nring;         // 2 nx + 2 ny, or the Turkel-Zwas pad (see ring_coord)
  int32_t pad_p, pad_q;  // Turkel-Zwas pad widths (0: the one-cell ring)
  int64_t ctrl_off;      // packed FP64 control offset (elements)
  int64_t traj_off;      // packed FP64 trajectory offset (elements)
  int64_t ncell() const { return int64_t(ny) * nx; }
};

}  // namespace dd4dvar

struct dd4dvar_plan {
  dd4dvar_model_desc model{};
  int32_t nspace = 0, ntime = 0, nsub = 0;
  std::vector<dd4dvar::BoxInfo> boxes;
  std::vector<int32_t> owner;       // [nlat*nlon] piece owning each core cell
  std::vector<int32_t> cover_sp;    // [nlat*nlon] spatial coverage count
  std::vector<int32_t> time_count;  // [nsteps+1]
  // per-subdomain ring maps, concatenated (offset ring_ptr[s])
  std::vector<int64_t> ring_ptr;
  std::vector<int32_t> halo_src, halo_off, halo_sign, halo_gcell;
  // per-subdomain box-cell coverage (offset cell_ptr[s])
  std::vector<int64_t> cell_ptr;
  std::vector<int32_t> cover_box;
  // overlap neighbours (CSR)
  std::vector<int64_t> nbr_ptr;
  std::vector<int32_t> nbr_idx;
  // observation bins (CSR of global observation indices)
  std::vector<int64_t> obs_ptr;
  std::vector<int32_t> obs_idx;
  int64_t ctrl_total = 0, traj_total = 0;
  // copies of the data descriptor
  std::vector<double> xb0, sigma_b;
  std::vector<int32_t> obs_step, obs_cell;
  std::vector<int8_t> obs_field;
  std::vector<double> obs_value, obs_sigma;
};

namespace dd4dvar {
// Builds a plan; on failure returns a status and fills err.
dd4dvar_status build_plan(const dd4dvar_model_desc* model,
                          const dd4dvar_partition_desc* part,
                          const dd4dvar_data_desc* data, dd4dvar_plan* plan,
                          std::string* err);
void set_thread_error(const std::string& msg);
const char* thread_error();
}  // namespace dd4dvar
