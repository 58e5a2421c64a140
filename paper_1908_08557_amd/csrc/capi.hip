// C ABI of the library (declared in include/cmhd.h): context, validation,
// workspace binding and the substage sequence of one RK3 step.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <algorithm>
#include <mutex>
#include <vector>

#include "launch.h"

using namespace cmhd;

// Reduction scratch of cmhd_cfl_dt_noalloc: the three maxima of the CFL
// kernel (3 x 8 bytes, padded), one copy per GPU held until the process ends.
// In host code this name is a stand-in, not a device address: the address of
// each GPU's copy is looked up once per device (init_noalloc_scratch) and only
// that pointer is handed to kernels.
static __device__ __align__(256) unsigned long long scratch[32];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned long long* g_scratch[kMaxDevices] = {};   // per device: &scratch on that GPU

// look up this device's copy of the scratch array (the device is current)
hipError_t init_noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[dev] = static_cast<unsigned long long*>(ptr);
  return e;
}
}  // namespace

struct cmhd_ctx {
  cmhd_grid grid;
  cmhd_params par;
  KParams kp;
  int dev = 0;            // the GPU current at init
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* W1 = nullptr;   // stage buffers
  double* W2 = nullptr;
  double* dF = nullptr;   // RK register
  double* uh = nullptr;   // driver u*      [2][ny][nx] (of the current substage)
  double* u0 = nullptr;   // driver snapshots [2][ny][nx] each, at snap_t0 and snap_t1
  double* u1 = nullptr;
  bool snap = false;
  double snap_t0 = 0.0, snap_t1 = 1.0;
  double* ah = nullptr;   // A_h* target    [2][ny][nx]
  double2* fft = nullptr; // Fourier scratch
  unsigned long long* red = nullptr;  // reduction scratch
  std::vector<double> nc_host;   // initial [ln rho0 | ln T0] profiles (Newtonian cooling)
  double* nc_dev = nullptr;      // their device copy in the workspace
  std::vector<double> z_host;    // plane heights z_k, k = -3..nz+2
  std::vector<double> zt_host;   // the z table of KParams::ztab (non-uniform grids)
  double* zt_dev = nullptr;
  KParams* kp_dev = nullptr;     // device copy of kp (read by the fused substage kernel)
  std::string err;
  // adjoint workspace
  char* aws = nullptr;
  double *Q = nullptr, *Qb = nullptr, *XB = nullptr, *dFB = nullptr, *RB = nullptr, *Gb = nullptr;
  bool profiling = false;
  // per timed kernel (CMHD_PROF_*): event pairs recorded and not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[2], ev_free;
  ~cmhd_ctx() {
    for (auto& v : ev_pending)
      for (auto& e : v) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }
};

namespace {

cmhd_status fail(cmhd_ctx* c, cmhd_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

cmhd_status hip_check(cmhd_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return CMHD_OK;
  return fail(c, CMHD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t state_elems(const cmhd_grid& g) {
  return size_t(NF) * size_t(g.nz + 2 * NG) * size_t(g.ny) * size_t(g.nx);
}

size_t ws_layout(const cmhd_ctx* c, size_t off[16]) {
  const size_t plane = size_t(c->grid.nx) * size_t(c->grid.ny);
  const size_t sb = align256(state_elems(c->grid) * sizeof(double));
  size_t o = 0;
  off[0] = o; o += sb;                                           // W1
  off[1] = o; o += sb;                                           // W2
  off[2] = o; o += sb;                                           // dF
  off[3] = o; o += align256(2 * plane * sizeof(double));         // uh
  off[4] = o; o += align256(2 * plane * sizeof(double));         // ah
  off[5] = o; o += align256(FFT_PLANES * plane * sizeof(double2));  // fft
  off[6] = o; o += 256;                                          // reductions
  off[7] = o;                                                    // (unused)
  off[8] = o; o += align256(2 * size_t(c->kp.nc_n) * sizeof(double));   // ln rho0, ln T0
  off[9] = o; o += align256(2 * plane * sizeof(double));         // driver snapshot 0
  off[10] = o; o += align256(2 * plane * sizeof(double));        // driver snapshot 1
  off[11] = o; o += align256(size_t(zt_size(c->kp)) * sizeof(double));  // z table
  off[12] = o; o += align256(sizeof(KParams));                   // parameter block
  return o;
}

// heights, metric and ghost distances of the z grid.  zin: the caller's
// heights (non-uniform grid) or NULL (uniform: z0 + k dz)
void fill_zgrid(cmhd_ctx* c, const double* zin) {
  KParams& p = c->kp;
  const int nz = p.nz, n = nz + 2 * NG;
  c->z_host.resize(n);
  for (int i = 0; i < n; ++i) c->z_host[i] = zin ? zin[i] : p.z0 + (i - NG) * p.dz;
  const double* z = c->z_host.data();
  p.stretched = zin != nullptr;
  p.dxy_min = std::fmin(p.dx, p.dy);
  c->zt_host.assign(size_t(zt_size(p)), 0.0);
  for (int i = 0; i < n; ++i) c->zt_host[i] = z[i];
  if (p.stretched) {
    p.z0 = z[NG];
    // z' and z'' at the interior planes from the sixth-order stencils in the
    // plane index applied to the heights
    for (int k = 0; k < nz; ++k) {
      const double* w = z + k + NG;
      const double zp = (45.0 * (w[1] - w[-1]) - 9.0 * (w[2] - w[-2]) + (w[3] - w[-3])) / 60.0;
      const double zpp =
          (-490.0 * w[0] + 270.0 * (w[1] + w[-1]) - 27.0 * (w[2] + w[-2]) + 2.0 * (w[3] + w[-3])) /
          180.0;
      c->zt_host[zt_c1(p) + k] = 1.0 / (60.0 * zp);
      c->zt_host[zt_c2(p) + k] = 1.0 / (180.0 * zp * zp);
      c->zt_host[zt_c3(p) + k] = -zpp / (60.0 * zp * zp * zp);
      c->zt_host[zt_zp(p) + k] = zp;
    }
  }
  const int kb = NG, kt = NG + nz - 1;
  for (int j = 1; j <= NG; ++j) {
    if (p.stretched) {
      p.dz_lo[j - 1] = z[kb - j + 1] - z[kb - j];
      p.dz_hi[j - 1] = z[kt + j] - z[kt + j - 1];
      p.pf_dist[0][j - 1] = -p.f_bot * (z[kb] - z[kb - j]);
      p.pf_dist[1][j - 1] = z[kt + j] - z[kt];
    } else {
      p.dz_lo[j - 1] = p.dz;
      p.dz_hi[j - 1] = p.dz;
      p.pf_dist[0][j - 1] = j * (-p.f_bot * p.dz);
      p.pf_dist[1][j - 1] = j * p.dz;
    }
  }
  p.ztab = nullptr;   // set when the workspace is bound
}

void fill_kparams(cmhd_ctx* c, const double* lnrho0_z) {
  const cmhd_grid& g = c->grid;
  const cmhd_params& q = c->par;
  KParams& p = c->kp;
  std::memset(&p, 0, sizeof(p));
  p.nx = g.nx;
  p.ny = g.ny;
  p.nz = g.nz;
  p.solar = g.zbc == CMHD_ZBC_SOLAR;
  p.splane = (long long)g.nx * g.ny;
  p.sfield = (long long)(g.nz + 2 * NG) * p.splane;
  p.dx = g.Lx / g.nx;
  p.dy = g.Ly / g.ny;
  p.dz = p.solar ? (g.z1 - g.z0) / (g.nz - 1) : (g.z1 - g.z0) / g.nz;
  p.z0 = g.z0;
  p.Lx = g.Lx;
  p.Ly = g.Ly;
  p.i60dx = 1.0 / (60.0 * p.dx);
  p.i60dy = 1.0 / (60.0 * p.dy);
  p.i60dz = 1.0 / (60.0 * p.dz);
  p.i180dx2 = 1.0 / (180.0 * p.dx * p.dx);
  p.i180dy2 = 1.0 / (180.0 * p.dy * p.dy);
  p.i180dz2 = 1.0 / (180.0 * p.dz * p.dz);
  p.gamma = q.gamma;
  p.R = q.R;
  p.mu0 = q.mu0;
  p.inv_mu0 = 1.0 / q.mu0;
  p.eta = q.eta;
  p.nu = q.nu;
  p.D_rho = q.D_rho;
  p.kappa0 = q.kappa0;
  p.g_z = q.g_z;
  p.cv = q.R / (q.gamma - 1.0);
  p.inv_cv = 1.0 / p.cv;
  p.gm1 = q.gamma - 1.0;
  for (int i = 0; i < 3; ++i) p.Bext[i] = q.Bext[i];
  p.B_floor2 = q.B_floor * q.B_floor;
  if (p.solar) {
    p.eta_s = q.eta_s;
    p.chi_s = q.chi_s;
    p.chi_rho = q.chi_rho;
    p.z_s = q.z_s;
    p.z_t = q.z_t;
    p.tau_u = q.tau_u;
    p.tau_A = q.tau_A;
  } else {
    p.z_s = 0.0;
    p.z_t = 1.0;
  }
  p.f_bot = q.f_bot;
  p.n_rad = q.n_rad;
  for (int i = 0; i < q.n_rad; ++i) {
    p.rad_lnT[i] = q.rad_lnT[i];
    p.rad_lnL[i] = q.rad_lnL[i];
  }
  for (int i = 0; i + 1 < q.n_rad; ++i)
    p.rad_slope[i] = (q.rad_lnL[i + 1] - q.rad_lnL[i]) / (q.rad_lnT[i + 1] - q.rad_lnT[i]);
  p.lnT_rad_lo = std::log(q.T_rad_lo);
  p.lnT_rad_hi = std::log(q.T_rad_hi);
  p.inv_dlnT_rad = 1.0 / (p.lnT_rad_hi - p.lnT_rad_lo);
  for (int i = 0; i < 4; ++i) p.lnrho0_bot[i] = lnrho0_z ? lnrho0_z[i] : 0.0;
  p.c_adv = q.c_adv;
  p.c_diff = q.c_diff;
  p.c_nudge = q.c_nudge;
  p.nc_tau = q.nc_tau;
  p.nc_dlr0 = q.nc_lnrho_magn - q.nc_lnrho_width;
  p.nc_dlrw = q.nc_lnrho_width;
  p.nc_z0 = q.nc_z_max - q.nc_z_width;
  p.nc_zw = q.nc_z_width;
  p.nc_dlr1 = p.nc_dlr0 + p.nc_dlrw;
  p.nc_dlrm = p.nc_dlr0 + 0.5 * p.nc_dlrw;
  p.nc_z1 = p.nc_z0 + p.nc_zw;
  p.nc_zm = p.nc_z0 + 0.5 * p.nc_zw;
  p.nc_pi_dlrw = q.nc_lnrho_width > 0.0 ? M_PI / q.nc_lnrho_width : 0.0;
  p.nc_pi_zw = q.nc_z_width > 0.0 ? M_PI / q.nc_z_width : 0.0;
  p.nc_lnrho_phot = lnrho0_z ? lnrho0_z[NG] : 0.0;
  p.nc_n = g.nz + 2 * NG;
  p.nc_tab = nullptr;   // set when the workspace is bound
}

double ramp(const cmhd_ctx* c, double t) {
  if (c->par.t_ramp <= 0.0) return 1.0;
  const double r = t / c->par.t_ramp;
  return r < 1.0 ? r : 1.0;
}

cmhd_status need_ws(cmhd_ctx* c) {
  if (!c->ws) return fail(c, CMHD_ESTATE, "no workspace bound (cmhd_bind_workspace)");
  return CMHD_OK;
}

cmhd_status do_fill(cmhd_ctx* c, double* state) {
  hipError_t e;
  if (c->kp.solar) {
    e = launch_fill_solar_columns(c->kp, state, c->stream);
    if (e == hipSuccess) e = launch_potential_ghosts(c->kp, state, c->fft, c->stream);
  } else {
    e = launch_fill_periodic_z(c->kp, state, c->stream);
  }
  return hip_check(c, e, "fill_ghosts launch");
}

// dt from the three maxima of the CFL kernel (speed / spacing or speed,
// diffusivity / spacing^2 or diffusivity, radiative rate) and the nudging rates
cmhd_status dt_from_maxima(cmhd_ctx* c, const unsigned long long h[3], double* dt_out) {
  double m[3];
  std::memcpy(m, h, sizeof(m));
  const KParams& p = c->kp;
  double dt;
  if (p.stretched) {
    // the kernel reduced speed / spacing and D / spacing^2 per plane
    dt = p.c_adv / m[0];
    if (m[1] > 0.0) dt = std::fmin(dt, p.c_diff / m[1]);
  } else {
    const double delta = std::fmin(p.dx, std::fmin(p.dy, p.dz));
    dt = p.c_adv * delta / m[0];
    if (m[1] > 0.0) dt = std::fmin(dt, p.c_diff * delta * delta / m[1]);
  }
  if (m[2] > 0.0) dt = std::fmin(dt, p.c_adv / m[2]);
  double tau = p.solar ? std::fmax(p.tau_u, p.tau_A) : 0.0;
  tau = std::fmax(tau, p.nc_tau);
  if (tau > 0.0) dt = std::fmin(dt, p.c_nudge / tau);
  if (std::isnan(m[0]) || std::isnan(m[1]) || std::isnan(m[2]))
    return fail(c, CMHD_ENONFINITE, "the state holds a non-finite value (CFL maxima are NaN)");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(c, CMHD_EDT, "the time step from the CFL limits is " + std::to_string(dt));
  *dt_out = dt;
  return CMHD_OK;
}

// the CFL maxima of a ghost-filled state reduced into red (3 values), copied
// to the host and turned into dt
cmhd_status cfl_reduce(cmhd_ctx* c, const double* state, unsigned long long* red,
                       double* dt_out) {
  hipError_t e = launch_cfl_max(c->kp, state, red, c->stream);
  if (e != hipSuccess) return hip_check(c, e, "cfl launch");
  unsigned long long h[3];
  e = hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "cfl copy");
  return dt_from_maxima(c, h, dt_out);
}

cmhd_status do_cfl(cmhd_ctx* c, double* state, double* dt_out) {
  cmhd_status st = do_fill(c, state);
  if (st != CMHD_OK) return st;
  return cfl_reduce(c, state, c->red, dt_out);
}

// event pair for one timed launch of kernel `which` (or none when not profiling)
hipError_t ev_begin(cmhd_ctx* c, std::pair<hipEvent_t, hipEvent_t>& ev) {
  ev = {nullptr, nullptr};
  if (!c->profiling) return hipSuccess;
  if (!c->ev_free.empty()) {
    ev = c->ev_free.back();
    c->ev_free.pop_back();
  } else {
    hipError_t e = hipEventCreate(&ev.first);
    if (e == hipSuccess) e = hipEventCreate(&ev.second);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(ev.first, c->stream);
}

hipError_t ev_end(cmhd_ctx* c, std::pair<hipEvent_t, hipEvent_t>& ev, int which) {
  if (!c->profiling) return hipSuccess;
  hipError_t e = hipEventRecord(ev.second, c->stream);
  c->ev_pending[which].push_back(ev);
  return e;
}

// the interior planes k0, k0+1 around height z and the weight a of k0+1
// (non-uniform grids); false outside the interior
bool plane_between(const cmhd_ctx* c, double z, int* k0, double* a) {
  const int nz = c->kp.nz;
  const double* zi = c->z_host.data() + NG;
  if (!(z >= zi[0]) || !(z <= zi[nz - 1])) return false;
  int k = int(std::upper_bound(zi, zi + nz, z) - zi) - 1;
  k = std::min(k, nz - 2);
  *k0 = k;
  *a = (z - zi[k]) / (zi[k + 1] - zi[k]);
  return true;
}

// the nudging target of a substage at time ts (snapshot pair: interpolated
// into the u* buffer; single target: nothing to do)
hipError_t driver_at(cmhd_ctx* c, double ts) {
  if (!c->kp.solar || !c->snap) return hipSuccess;
  const double w = std::min(1.0, std::max(0.0, (ts - c->snap_t0) / (c->snap_t1 - c->snap_t0)));
  return launch_driver_interp(c->kp, c->u0, c->u1, w, c->uh, c->stream);
}

// One substage s from src to dst with the stage arguments a at the stage
// time ts: the boundary work (ghost fill of src, the driver target at ts, the
// nudged u_h ghost rows, which touch no plane of the fused kernel), then the
// fused stencil/RHS/RK kernel.  Each part is timed when profiling is on.
cmhd_status substage(cmhd_ctx* c, int s, double* src, double* dst, double* dF,
                     const StageArgs& a, double ts) {
  std::pair<hipEvent_t, hipEvent_t> ev;
  hipError_t e = ev_begin(c, ev);
  if (e != hipSuccess) return hip_check(c, e, "profiling event");
  cmhd_status st = do_fill(c, src);
  if (st != CMHD_OK) return st;
  e = driver_at(c, ts);
  if (e == hipSuccess && c->kp.solar)
    e = launch_ghost_rows(c->kp, src, dst, dF, c->uh, a, s > 0, s < 2, c->stream);
  if (e == hipSuccess) e = ev_end(c, ev, CMHD_PROF_GHOSTS);
  if (e == hipSuccess) e = ev_begin(c, ev);
  if (e == hipSuccess)
    e = launch_substage(c->kp, c->kp_dev, c->grid.prec, s, src, dst, dF, c->uh, c->ah, a,
                        c->stream);
  if (e == hipSuccess) e = ev_end(c, ev, CMHD_PROF_SUBSTAGE);
  return hip_check(c, e, "substage launch");
}

}  // namespace

extern "C" {

cmhd_status cmhd_init_grid_z(const cmhd_grid* grid, const cmhd_params* params, const double* z,
                             const double* lnrho0_z, const double* lnT0_z, void* stream,
                             cmhd_ctx** out) {
  if (!out) return CMHD_EINVAL;
  *out = nullptr;
  if (!grid || !params) return CMHD_EINVAL;
  const cmhd_grid& g = *grid;
  const cmhd_params& q = *params;
  const bool solar = g.zbc == CMHD_ZBC_SOLAR;
  std::string why;
  if (!pow2(g.nx) || !pow2(g.ny) || g.nx < 16 || g.ny < 16 || g.nx > 1024 || g.ny > 1024)
    why = "nx, ny must be powers of two in [16, 1024]";
  else if (g.nz < 8)
    why = "nz must be >= 8";
  else if (g.zbc != CMHD_ZBC_PERIODIC && g.zbc != CMHD_ZBC_SOLAR)
    why = "zbc must be CMHD_ZBC_PERIODIC or CMHD_ZBC_SOLAR";
  else if (g.prec != CMHD_FP64 && g.prec != CMHD_FP32_SPLIT)
    why = "prec must be CMHD_FP64 or CMHD_FP32_SPLIT";
  else if (!(g.Lx > 0) || !(g.Ly > 0) || (!z && !(g.z1 > g.z0)))
    why = "domain lengths must be positive";
  else if (!(q.gamma > 1.0) || !(q.R > 0) || !(q.mu0 > 0))
    why = "gamma > 1, R > 0 and mu0 > 0 are required";
  else if (q.eta < 0 || q.nu < 0 || q.D_rho < 0 || q.kappa0 < 0)
    why = "diffusivities must be non-negative";
  else if (q.n_rad < 0 || q.n_rad == 1 || q.n_rad > CMHD_MAX_RAD)
    why = "n_rad must be 0 or in [2, 16]";
  else if (q.n_rad > 0 && !(q.T_rad_hi > q.T_rad_lo && q.T_rad_lo > 0))
    why = "0 < T_rad_lo < T_rad_hi is required";
  else if (solar && !(q.z_t > q.z_s))
    why = "z_t > z_s is required";
  else if (solar && !lnrho0_z)
    why = "solar mode needs the ln rho0(z) profile";
  else if (!(q.nc_tau >= 0.0))
    why = "nc_tau must be non-negative";
  else if (q.nc_tau > 0.0 && (!lnrho0_z || !lnT0_z))
    why = "the Newtonian cooling needs the ln rho0(z) and ln T0(z) profiles";
  else if (q.nc_tau > 0.0 && g.nz + 2 * NG > CMHD_MAX_NC_TABLE)
    why = "the Newtonian cooling supports nz + 6 <= CMHD_MAX_NC_TABLE";
  else if (q.nc_tau > 0.0 && !(q.nc_lnrho_width > 0.0 && q.nc_z_width > 0.0 &&
                               q.nc_lnrho_magn >= q.nc_lnrho_width))
    why = "Newtonian cooling cutoffs: widths > 0 and nc_lnrho_magn >= nc_lnrho_width";
  for (int i = 0; why.empty() && i + 1 < q.n_rad; ++i)
    if (!(q.rad_lnT[i + 1] > q.rad_lnT[i])) why = "rad_lnT must increase";
  for (int i = 0; why.empty() && q.nc_tau > 0.0 && i + 1 < g.nz + 2 * NG; ++i)
    if (!(lnrho0_z[i + 1] < lnrho0_z[i]))
      why = "the Newtonian cooling needs ln rho0(z) to decrease strictly with height";
  if (why.empty() && z && !solar) why = "a non-uniform z grid needs the solar boundaries";
  for (int i = 0; why.empty() && z && i < g.nz + 2 * NG; ++i)
    if (!std::isfinite(z[i]) || (i > 0 && !(z[i] > z[i - 1])))
      why = "the heights z_k must be finite and increase strictly";
  if (!why.empty()) {
    std::fprintf(stderr, "cmhd_init_grid: %s\n", why.c_str());
    return CMHD_EINVAL;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    std::fprintf(stderr, "cmhd_init_grid: no HIP device\n");
    return CMHD_EDEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    std::fprintf(stderr, "cmhd_init_grid: device is %s, the library is built for gfx950\n",
                 prop.gcnArchName);
    return CMHD_EDEVICE;
  }
  if (init_noalloc_scratch(dev) != hipSuccess) {
    std::fprintf(stderr, "cmhd_init_grid: no address for the library's device scratch\n");
    return CMHD_EDEVICE;
  }
  cmhd_ctx* c = new cmhd_ctx();
  c->grid = g;
  c->par = q;
  c->dev = dev;
  c->stream = (hipStream_t)stream;
  fill_kparams(c, lnrho0_z);
  fill_zgrid(c, z);
  {
    const int n = g.nz + 2 * NG;
    c->nc_host.assign(2 * size_t(n), 0.0);
    for (int i = 0; i < n; ++i) {
      c->nc_host[i] = lnrho0_z ? lnrho0_z[i] : 0.0;
      c->nc_host[n + i] = lnT0_z ? lnT0_z[i] : 0.0;
    }
  }
  *out = c;
  return CMHD_OK;
}

cmhd_status cmhd_init_grid(const cmhd_grid* grid, const cmhd_params* params,
                           const double* lnrho0_z, const double* lnT0_z, void* stream,
                           cmhd_ctx** out) {
  return cmhd_init_grid_z(grid, params, nullptr, lnrho0_z, lnT0_z, stream, out);
}

size_t cmhd_state_elems(const cmhd_ctx* c) { return c ? state_elems(c->grid) : 0; }

size_t cmhd_workspace_bytes(const cmhd_ctx* c) {
  if (!c) return 0;
  size_t off[16];
  return ws_layout(c, off);
}

cmhd_status cmhd_bind_workspace(cmhd_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return CMHD_EINVAL;
  size_t off[16];
  const size_t need = ws_layout(c, off);
  if (!dev_ptr) return fail(c, CMHD_EINVAL, "workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0)
    return fail(c, CMHD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(c, CMHD_EWORKSPACE,
                "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(need));
  c->ws = static_cast<char*>(dev_ptr);
  c->ws_bytes = bytes;
  c->W1 = reinterpret_cast<double*>(c->ws + off[0]);
  c->W2 = reinterpret_cast<double*>(c->ws + off[1]);
  c->dF = reinterpret_cast<double*>(c->ws + off[2]);
  c->uh = reinterpret_cast<double*>(c->ws + off[3]);
  c->ah = reinterpret_cast<double*>(c->ws + off[4]);
  c->fft = reinterpret_cast<double2*>(c->ws + off[5]);
  c->red = reinterpret_cast<unsigned long long*>(c->ws + off[6]);
  c->nc_dev = reinterpret_cast<double*>(c->ws + off[8]);
  c->u0 = reinterpret_cast<double*>(c->ws + off[9]);
  c->u1 = reinterpret_cast<double*>(c->ws + off[10]);
  c->snap = false;
  c->zt_dev = reinterpret_cast<double*>(c->ws + off[11]);
  c->kp.ztab = c->zt_dev;
  c->kp.nc_tab = c->nc_dev;
  c->kp_dev = reinterpret_cast<KParams*>(c->ws + off[12]);
  // driver targets start at zero; the stage buffers are fully written before use
  const size_t plane = size_t(c->grid.nx) * size_t(c->grid.ny);
  hipError_t e = hipMemsetAsync(c->uh, 0, 2 * plane * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ah, 0, 2 * plane * sizeof(double), c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->nc_dev, c->nc_host.data(), c->nc_host.size() * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->zt_dev, c->zt_host.data(), c->zt_host.size() * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->kp_dev, &c->kp, sizeof(KParams), hipMemcpyHostToDevice, c->stream);
  // the tables are read from host vectors that outlive the copies
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return hip_check(c, e, "workspace clear");
}

cmhd_status cmhd_set_stream(cmhd_ctx* c, void* stream) {
  if (!c) return CMHD_EINVAL;
  c->stream = (hipStream_t)stream;
  return CMHD_OK;
}

cmhd_status cmhd_set_driver(cmhd_ctx* c, const double* uh, const double* bz, const double* ah) {
  if (!c) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  if (!uh) return fail(c, CMHD_EINVAL, "uh is NULL");
  if (bz && ah) return fail(c, CMHD_EINVAL, "give bz or ah, not both");
  const size_t plane = size_t(c->grid.nx) * size_t(c->grid.ny);
  hipError_t e = hipMemcpyAsync(c->uh, uh, 2 * plane * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream);
  if (e != hipSuccess) return hip_check(c, e, "driver copy");
  c->snap = false;
  if (ah) {
    e = hipMemcpyAsync(c->ah, ah, 2 * plane * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_check(c, e, "driver copy");
  }
  if (bz) {
    // balanced flux (Sect. 2.1): |sum B_z| <= 1e-12 sum |B_z|
    double* red2 = reinterpret_cast<double*>(c->red) + 4;
    e = hipMemsetAsync(red2, 0, 2 * sizeof(double), c->stream);
    if (e == hipSuccess) e = launch_sum_abs(c->kp, bz, red2, c->stream);
    double h[2] = {0, 0};
    if (e == hipSuccess)
      e = hipMemcpyAsync(h, red2, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "net flux");
    if (std::fabs(h[0]) > 1e-12 * h[1])
      return fail(c, CMHD_EINVAL, "B_z has a net flux (sum " + std::to_string(h[0]) + ")");
    e = launch_ah_from_bz(c->kp, bz, c->ah, c->fft, c->stream);
    if (e != hipSuccess) return hip_check(c, e, "A_h* from B_z");
  }
  return CMHD_OK;
}

cmhd_status cmhd_set_driver_snapshots(cmhd_ctx* c, const double* uh0, double t0,
                                      const double* uh1, double t1) {
  if (!c) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  if (!uh0 || !uh1) return fail(c, CMHD_EINVAL, "a driver snapshot is NULL");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 > t0))
    return fail(c, CMHD_EINVAL, "snapshot times must be finite with t1 > t0");
  const size_t bytes = 2 * size_t(c->grid.nx) * size_t(c->grid.ny) * sizeof(double);
  hipError_t e = hipMemcpyAsync(c->u0, uh0, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->u1, uh1, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_check(c, e, "driver snapshot copy");
  c->snap = true;
  c->snap_t0 = t0;
  c->snap_t1 = t1;
  return CMHD_OK;
}

cmhd_status cmhd_fill_ghosts(cmhd_ctx* c, double* state, double t) {
  (void)t;
  if (!c || !state) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  return do_fill(c, state);
}

cmhd_status cmhd_cfl_dt(cmhd_ctx* c, double* state, double* dt_out) {
  if (!c || !state || !dt_out) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  return do_cfl(c, state, dt_out);
}

cmhd_status cmhd_cfl_dt_noalloc(cmhd_ctx* c, const double* state, double* dt_out) {
  if (!c || !state || !dt_out) return CMHD_EINVAL;
  if (c->kp.stretched && !c->ws)
    return fail(c, CMHD_ESTATE, "a non-uniform z grid needs the bound workspace (its z table)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != c->dev)
    return fail(c, CMHD_ESTATE, "the context's GPU is not the current device");
  unsigned long long* red = g_scratch[c->dev];
  if (!red) return fail(c, CMHD_ESTATE, "no device scratch for this GPU");
  return cfl_reduce(c, state, red, dt_out);
}

cmhd_status cmhd_rk3_step(cmhd_ctx* c, double* state, double* t, double dt, double* dt_used) {
  if (!c || !state || !t) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  if (!(dt > 0.0)) {
    st = do_cfl(c, state, &dt);
    if (st != CMHD_OK) return st;
  }
  double* src[3] = {state, c->W1, c->W2};
  double* dst[3] = {c->W1, c->W2, state};
  for (int s = 0; s < 3; ++s) {
    const double ts = *t + RK_C[s] * dt;
    StageArgs a{RK_ALPHA[s], RK_BETA[s], dt, ramp(c, ts)};
    st = substage(c, s, src[s], dst[s], c->dF, a, ts);
    if (st != CMHD_OK) return st;
  }
  *t += dt;
  if (dt_used) *dt_used = dt;
  return CMHD_OK;
}

cmhd_status cmhd_eval_rhs(cmhd_ctx* c, double* state, double t, double* rhs) {
  if (!c || !state || !rhs) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  // one substage with alpha = 0, beta = 0, dt = 1: dF = RHS, f_next = f (into W1)
  StageArgs a{0.0, 0.0, 1.0, ramp(c, t)};
  return substage(c, 0, state, c->W1, rhs, a, t);
}

cmhd_status cmhd_get_fields(cmhd_ctx* c, const double* state, unsigned mask, double* dst,
                            int dst_on_host, int with_ghosts) {
  if (!c || !state || !dst) return CMHD_EINVAL;
  if (mask == 0 || mask > 0xFFu) return fail(c, CMHD_EINVAL, "mask selects no valid field");
  const size_t plane = size_t(c->grid.nx) * size_t(c->grid.ny);
  const size_t nzc = with_ghosts ? size_t(c->grid.nz + 2 * NG) : size_t(c->grid.nz);
  const size_t off = with_ghosts ? 0 : NG * plane;
  const size_t per = nzc * plane;
  const size_t sfield = size_t(c->grid.nz + 2 * NG) * plane;
  const hipMemcpyKind kind = dst_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  size_t o = 0;
  for (int f = 0; f < NF; ++f) {
    if (!(mask & (1u << f))) continue;
    hipError_t e = hipMemcpyAsync(dst + o, state + f * sfield + off, per * sizeof(double), kind,
                                  c->stream);
    if (e != hipSuccess) return hip_check(c, e, "get_fields copy");
    o += per;
  }
  if (dst_on_host) return hip_check(c, hipStreamSynchronize(c->stream), "get_fields sync");
  return CMHD_OK;
}

cmhd_status cmhd_set_fields(cmhd_ctx* c, double* state, unsigned mask, const double* src,
                            int src_on_host, int with_ghosts) {
  if (!c || !state || !src) return CMHD_EINVAL;
  if (mask == 0 || mask > 0xFFu) return fail(c, CMHD_EINVAL, "mask selects no valid field");
  const size_t plane = size_t(c->grid.nx) * size_t(c->grid.ny);
  const size_t nzc = with_ghosts ? size_t(c->grid.nz + 2 * NG) : size_t(c->grid.nz);
  const size_t off = with_ghosts ? 0 : NG * plane;
  const size_t per = nzc * plane;
  const size_t sfield = size_t(c->grid.nz + 2 * NG) * plane;
  const hipMemcpyKind kind = src_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  size_t o = 0;
  for (int f = 0; f < NF; ++f) {
    if (!(mask & (1u << f))) continue;
    hipError_t e = hipMemcpyAsync(state + f * sfield + off, src + o, per * sizeof(double), kind,
                                  c->stream);
    if (e != hipSuccess) return hip_check(c, e, "set_fields copy");
    o += per;
  }
  if (src_on_host) return hip_check(c, hipStreamSynchronize(c->stream), "set_fields sync");
  return CMHD_OK;
}

cmhd_status cmhd_bz_plane(cmhd_ctx* c, const double* state, double z, double* dst) {
  if (!c || !state || !dst) return CMHD_EINVAL;
  const KParams& p = c->kp;
  if (!p.stretched) {
    if (!(z >= p.z0) || !(z <= p.z0 + (p.nz - 1) * p.dz))
      return fail(c, CMHD_EINVAL, "z outside the interior");
    return hip_check(c, launch_bz_plane(p, state, z, dst, c->stream), "bz_plane launch");
  }
  int k0;
  double a;
  if (!plane_between(c, z, &k0, &a)) return fail(c, CMHD_EINVAL, "z outside the interior");
  return hip_check(c, launch_bz_plane_k(p, state, k0, a, dst, c->stream), "bz_plane launch");
}

cmhd_status cmhd_check_finite(cmhd_ctx* c, const double* state) {
  if (!c || !state) return CMHD_EINVAL;
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  int* flag = reinterpret_cast<int*>(c->red + 6);
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), c->stream);
  if (e == hipSuccess) e = launch_finite_check(c->kp, state, flag, c->stream);
  int h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "finite check");
  return h ? fail(c, CMHD_ENONFINITE, "state holds a non-finite value") : CMHD_OK;
}

namespace {

size_t adj_layout(const cmhd_ctx* c, size_t off[8]) {
  const size_t nzone = size_t(c->grid.nx) * size_t(c->grid.ny) * size_t(c->grid.nz);
  const size_t qb = align256(NQ_POINT * nzone * sizeof(double));
  const size_t sb = align256(state_elems(c->grid) * sizeof(double));
  size_t o = 0;
  off[0] = o; o += qb;   // Q
  off[1] = o; o += qb;   // Qbar / dQ
  off[2] = o; o += sb;   // XB / dX
  off[3] = o; o += sb;   // dFB / dDF
  off[4] = o; o += sb;   // RB / dR
  off[5] = o; o += sb;   // Gbar
  return o;
}

cmhd_status need_adj(cmhd_ctx* c) {
  cmhd_status st = need_ws(c);
  if (st != CMHD_OK) return st;
  if (!c->aws) return fail(c, CMHD_ESTATE, "no adjoint workspace bound");
  return CMHD_OK;
}

// forward substage s from src to dst (fills the ghosts of src first)
cmhd_status fwd_stage(cmhd_ctx* c, int s, double* src, double* dst, double t, double dt) {
  const double ts = t + RK_C[s] * dt;
  StageArgs a{RK_ALPHA[s], RK_BETA[s], dt, ramp(c, ts)};
  return substage(c, s, src, dst, c->dF, a, ts);
}

}  // namespace

size_t cmhd_adjoint_workspace_bytes(const cmhd_ctx* c) {
  if (!c) return 0;
  size_t off[8];
  return adj_layout(c, off);
}

cmhd_status cmhd_bind_adjoint_workspace(cmhd_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return CMHD_EINVAL;
  size_t off[8];
  const size_t need = adj_layout(c, off);
  if (!dev_ptr) return fail(c, CMHD_EINVAL, "adjoint workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0)
    return fail(c, CMHD_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (bytes < need) return fail(c, CMHD_EWORKSPACE, "adjoint workspace too small");
  c->aws = static_cast<char*>(dev_ptr);
  c->Q = reinterpret_cast<double*>(c->aws + off[0]);
  c->Qb = reinterpret_cast<double*>(c->aws + off[1]);
  c->XB = reinterpret_cast<double*>(c->aws + off[2]);
  c->dFB = reinterpret_cast<double*>(c->aws + off[3]);
  c->RB = reinterpret_cast<double*>(c->aws + off[4]);
  c->Gb = reinterpret_cast<double*>(c->aws + off[5]);
  return CMHD_OK;
}

cmhd_status cmhd_rk3_step_jvp(cmhd_ctx* c, double* x, double t, double dt, const double* dx,
                              const double* duh, double* dy) {
  if (!c || !x || !dx || !dy || !(dt > 0.0)) return CMHD_EINVAL;
  cmhd_status st = need_adj(c);
  if (st != CMHD_OK) return st;
  if (duh && c->snap)
    return fail(c, CMHD_EINVAL, "no driver perturbation with a snapshot pair as driver");
  const KParams& p = c->kp;
  hipStream_t s = c->stream;
  const size_t sbytes = state_elems(c->grid) * sizeof(double);
  double* X[3] = {x, c->W1, c->W2};
  double* DX = c->XB;
  double* DDF = c->dFB;
  double* DR = c->RB;
  hipError_t e = launch_copy_state_entries(p, dx, DX, s);
  if (e == hipSuccess) e = hipMemsetAsync(DDF, 0, sbytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(DR, 0, sbytes, s);
  if (e != hipSuccess) return hip_check(c, e, "jvp init");
  st = do_fill(c, x);
  if (st != CMHD_OK) return st;
  for (int k = 0; k < 3; ++k) {
    const double rs = ramp(c, t + RK_C[k] * dt);
    e = driver_at(c, t + RK_C[k] * dt);
    if (e == hipSuccess) e = launch_fill_lin(p, X[k], DX, c->fft, s);
    if (e == hipSuccess) e = launch_point_q(p, X[k], c->Q, s);
    if (e == hipSuccess) e = launch_point_q(p, DX, c->Qb, s);
    if (e == hipSuccess) e = launch_point_jvp(p, c->Q, c->Qb, c->uh, c->ah, duh, rs, DR, s);
    if (e == hipSuccess && p.solar) e = launch_ghost_rows_jvp(p, DX, duh, rs, DR, s);
    if (e == hipSuccess) e = launch_tlm_combine(p, RK_ALPHA[k], RK_BETA[k], dt, DR, DDF, DX, s);
    if (e != hipSuccess) return hip_check(c, e, "jvp substage");
    if (k < 2) {
      st = fwd_stage(c, k, X[k], X[k + 1], t, dt);
      if (st != CMHD_OK) return st;
      st = do_fill(c, X[k + 1]);
      if (st != CMHD_OK) return st;
    }
  }
  return hip_check(c, launch_copy_state_entries(p, DX, dy, s), "jvp output");
}

cmhd_status cmhd_rk3_step_vjp(cmhd_ctx* c, double* x, double t, double dt, const double* ybar,
                              double* xbar, double* uhbar) {
  if (!c || !x || !ybar || !xbar || !(dt > 0.0)) return CMHD_EINVAL;
  cmhd_status st = need_adj(c);
  if (st != CMHD_OK) return st;
  if (uhbar && c->snap)
    return fail(c, CMHD_EINVAL, "no driver cotangent with a snapshot pair as driver");
  const KParams& p = c->kp;
  hipStream_t s = c->stream;
  const size_t sbytes = state_elems(c->grid) * sizeof(double);
  double* X[3] = {x, c->W1, c->W2};
  // forward substages 1 and 2: the linearisation points, ghost-filled
  st = fwd_stage(c, 0, X[0], X[1], t, dt);
  if (st == CMHD_OK) st = fwd_stage(c, 1, X[1], X[2], t, dt);
  if (st == CMHD_OK) st = do_fill(c, X[2]);
  if (st != CMHD_OK) return st;
  // uhbar may be NULL: accumulate into the Gbar buffer's first planes then drop
  double* uhb = uhbar ? uhbar : c->Gb;
  hipError_t e = launch_copy_state_entries(p, ybar, c->XB, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->dFB, 0, sbytes, s);
  if (e != hipSuccess) return hip_check(c, e, "vjp init");
  for (int k = 2; k >= 0; --k) {
    const double rs = ramp(c, t + RK_C[k] * dt);
    e = driver_at(c, t + RK_C[k] * dt);
    if (e == hipSuccess) e = launch_adj_combine(p, RK_ALPHA[k], RK_BETA[k], dt, c->XB, c->dFB, c->RB, s);
    if (e == hipSuccess) e = launch_point_q(p, X[k], c->Q, s);
    if (e == hipSuccess) e = launch_point_vjp(p, c->Q, c->RB, c->uh, c->ah, rs, c->Qb, uhb, s);
    if (e == hipSuccess) e = launch_stencil_T(p, c->Qb, c->Gb, s);
    if (e == hipSuccess) e = launch_fold_ghosts_T(p, X[k], c->Gb, c->XB, c->fft, s);
    if (e == hipSuccess && p.solar) e = launch_ghost_rows_vjp(p, c->RB, rs, c->XB, uhb, s);
    if (e != hipSuccess) return hip_check(c, e, "vjp substage");
    if (!uhbar) {   // the scratch use of Gbar must not leak into the next substage
      e = hipMemsetAsync(c->Gb, 0, 2 * size_t(p.splane) * sizeof(double), s);
      if (e != hipSuccess) return hip_check(c, e, "vjp scratch");
    }
  }
  return hip_check(c, launch_copy_state_entries(p, c->XB, xbar, s), "vjp output");
}

cmhd_status cmhd_bz_plane_vjp(cmhd_ctx* c, double z, const double* bzbar, double* xbar) {
  if (!c || !bzbar || !xbar) return CMHD_EINVAL;
  const KParams& p = c->kp;
  if (!p.stretched) {
    if (!(z >= p.z0) || !(z <= p.z0 + (p.nz - 1) * p.dz))
      return fail(c, CMHD_EINVAL, "z outside the interior");
    return hip_check(c, launch_bz_plane_vjp(p, z, bzbar, xbar, c->stream), "bz_plane_vjp launch");
  }
  int k0;
  double a;
  if (!plane_between(c, z, &k0, &a)) return fail(c, CMHD_EINVAL, "z outside the interior");
  return hip_check(c, launch_bz_plane_vjp_k(p, k0, a, bzbar, xbar, c->stream),
                   "bz_plane_vjp launch");
}

cmhd_status cmhd_profile_enable(cmhd_ctx* c, int enable) {
  if (!c) return CMHD_EINVAL;
  c->profiling = enable != 0;
  return CMHD_OK;
}

cmhd_status cmhd_profile_read(cmhd_ctx* c, int which, double* ms, int* launches) {
  if (!c || !ms || !launches) return CMHD_EINVAL;
  if (which != CMHD_PROF_SUBSTAGE && which != CMHD_PROF_GHOSTS)
    return fail(c, CMHD_EINVAL, "unknown kernel selector");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "profile sync");
  double sum = 0.0;
  for (auto& ev : c->ev_pending[which]) {
    float t = 0.0f;
    e = hipEventElapsedTime(&t, ev.first, ev.second);
    if (e != hipSuccess) return hip_check(c, e, "event elapsed");
    sum += t;
    c->ev_free.push_back(ev);
  }
  *launches = int(c->ev_pending[which].size());
  c->ev_pending[which].clear();
  *ms = sum;
  return CMHD_OK;
}

const char* cmhd_last_error(const cmhd_ctx* c) { return c ? c->err.c_str() : "null context"; }

void cmhd_destroy(cmhd_ctx* c) { delete c; }

}  // extern "C"
