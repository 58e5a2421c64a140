// Photospheric granulation driver (Sect. 2.3, eqs. 1-4): the granule
// population is host bookkeeping (births, deaths, advection: sequential by
// nature), the velocity snapshot is computed on the GPU (tile-culled render of
// the granular field, rotational part through 2-D FFTs, rms rescaling).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "launch.h"

using namespace cmhd;

struct cmhd_gran {
  cmhd_gran_params p;
  hipStream_t stream = nullptr;
  double dx = 0.0, dy = 0.0;
  int capacity = 0;
  // living granules, rows (x, y, t0, T, vmax, tmax) in birth order
  std::vector<double> tab;
  bool has_last = false;
  double t_last = 0.0;
  bool dirty = false;          // the device copy of the table is out of date
  // free-pixel flags and a Fenwick tree over them (k-th free pixel)
  std::vector<uint8_t> free_px;
  std::vector<int> fen;
  // device workspace
  char* ws = nullptr;
  double* dtab = nullptr;      // [capacity][6]
  double2* spec = nullptr;     // [2][ny][nx]
  double* part = nullptr;      // [2][kRedBlocks] partial sums, then the scale
  std::string err;
};

namespace {

constexpr int kTile = 16;
constexpr int kRedBlocks = 256;
constexpr int kRow = 6;

cmhd_status gfail(cmhd_gran* g, cmhd_status s, const std::string& m) {
  if (g) g->err = m;
  return s;
}

size_t galign(size_t b) { return (b + 255) & ~size_t(255); }

size_t gran_layout(const cmhd_gran* g, size_t off[3]) {
  const size_t plane = size_t(g->p.nx) * size_t(g->p.ny);
  size_t o = 0;
  off[0] = o; o += galign(size_t(g->capacity) * kRow * sizeof(double));
  off[1] = o; o += galign(2 * plane * sizeof(double2));
  off[2] = o; o += galign((2 * kRedBlocks + 8) * sizeof(double));
  return o;
}

// ---------------------------------------------------------------------------
// host bookkeeping (exact decisions: no contraction of products and sums)
// ---------------------------------------------------------------------------

double pdelta(double d, double L) {
#pragma clang fp contract(off)
  return d - L * std::floor(d / L + 0.5);
}

void fen_build(cmhd_gran* g) {
  const int n = int(g->free_px.size());
  g->fen.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int idx = i + 1;
    g->fen[idx] += g->free_px[i];
    const int par = idx + (idx & -idx);
    if (par <= n) g->fen[par] += g->fen[idx];
  }
}

void fen_add(cmhd_gran* g, int i, int d) {
  const int n = int(g->free_px.size());
  for (int idx = i + 1; idx <= n; idx += idx & -idx) g->fen[idx] += d;
}

// index of the k-th (0-based) free pixel in raster order
int fen_select(const cmhd_gran* g, int k) {
  const int n = int(g->free_px.size());
  int pos = 0, step = 1;
  while (step * 2 <= n) step *= 2;
  for (; step > 0; step >>= 1) {
    if (pos + step <= n && g->fen[pos + step] <= k) {
      pos += step;
      k -= g->fen[pos];
    }
  }
  return pos;   // pixel index (0-based) = pos
}

// mark the pixels closer than r_excl to (xc, yc) as taken; with the Fenwick
// tree kept in step when `tree` is set
void stamp(cmhd_gran* g, double xc, double yc, bool tree) {
#pragma clang fp contract(off)
  const int nx = g->p.nx, ny = g->p.ny;
  const double r2 = g->p.r_excl * g->p.r_excl;
  const int mx = int(std::ceil(g->p.r_excl / g->dx)) + 1;
  const int my = int(std::ceil(g->p.r_excl / g->dy)) + 1;
  const int ic = int(std::floor(xc / g->dx)), jc = int(std::floor(yc / g->dy));
  const bool allx = 2 * mx + 2 >= nx, ally = 2 * my + 2 >= ny;
  const int i0 = allx ? 0 : ic - mx, i1 = allx ? nx - 1 : ic + 1 + mx;
  const int j0 = ally ? 0 : jc - my, j1 = ally ? ny - 1 : jc + 1 + my;
  for (int jj = j0; jj <= j1; ++jj) {
    const int j = ((jj % ny) + ny) % ny;
    const double dy = pdelta(double(j) * g->dy - yc, g->p.Ly);
    for (int ii = i0; ii <= i1; ++ii) {
      const int i = ((ii % nx) + nx) % nx;
      const double dx = pdelta(double(i) * g->dx - xc, g->p.Lx);
      const double d2 = dy * dy + dx * dx;
      const size_t q = size_t(j) * nx + i;
      if (d2 < r2 && g->free_px[q]) {
        g->free_px[q] = 0;
        if (tree) fen_add(g, int(q), -1);
      }
    }
  }
}

double bilinear(const double* v, const cmhd_gran* g, double x, double y) {
#pragma clang fp contract(off)
  const int nx = g->p.nx, ny = g->p.ny;
  const double fx = x / g->dx, fy = y / g->dy;
  const double fi = std::floor(fx), fj = std::floor(fy);
  const double a = fx - fi, b = fy - fj;
  const int i0 = ((int(fi) % nx) + nx) % nx, j0 = ((int(fj) % ny) + ny) % ny;
  const int i1 = (i0 + 1) % nx, j1 = (j0 + 1) % ny;
  const double v00 = v[size_t(j0) * nx + i0], v01 = v[size_t(j0) * nx + i1];
  const double v10 = v[size_t(j1) * nx + i0], v11 = v[size_t(j1) * nx + i1];
  return (1.0 - a) * (1.0 - b) * v00 + a * (1.0 - b) * v01 + (1.0 - a) * b * v10 + a * b * v11;
}

double wrap(double x, double L) {
#pragma clang fp contract(off)
  return x - L * std::floor(x / L);
}

// ---------------------------------------------------------------------------
// device: the velocity snapshot
// ---------------------------------------------------------------------------

struct GranDev {
  int nx, ny;
  double Lx, Ly, dx, dy, r_gran, r_lane, inv_lane_w, f_rot;
};

__device__ __forceinline__ double dpdelta(double d, double L) {
  return d - L * floor(d / L + 0.5);
}

// One block per 16 x 16 pixel tile.  Granules are taken 256 at a time: each
// thread tests one against the tile (box test, conservative), the hits are
// compacted in order into LDS, then every pixel sums over the hits.
__global__ __launch_bounds__(256) void k_gran_render(const double* __restrict__ tab, int n,
                                                     double t, GranDev g,
                                                     double* __restrict__ v) {
  __shared__ double sx[256], sy[256], sa[256];
  __shared__ int wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = blockIdx.x * kTile + (tid & 15), j = blockIdx.y * kTile + (tid >> 4);
  const double px = double(i) * g.dx, py = double(j) * g.dy;
  const double cx = (double(blockIdx.x * kTile) + 7.5) * g.dx;
  const double cy = (double(blockIdx.y * kTile) + 7.5) * g.dy;
  const double hx = 8.5 * g.dx + g.r_lane, hy = 8.5 * g.dy + g.r_lane;
  const double rl2 = g.r_lane * g.r_lane;
  double vx = 0.0, vy = 0.0;
  for (int base = 0; base < n; base += 256) {
    const int q = base + tid;
    bool hit = false;
    double gx = 0.0, gy = 0.0, amp = 0.0;
    if (q < n) {
      const double* r = tab + size_t(q) * kRow;
      gx = r[0];
      gy = r[1];
      const double a = (t - r[2] - r[5]) / r[3];
      amp = r[4] * exp(-(a * a));
      hit = fabs(dpdelta(gx - cx, g.Lx)) <= hx && fabs(dpdelta(gy - cy, g.Ly)) <= hy;
    }
    const unsigned long long m = __ballot(hit);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();   // the previous chunk's hits have been read
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wave ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (hit) {
      sx[off + before] = gx;
      sy[off + before] = gy;
      sa[off + before] = amp;
    }
    __syncthreads();
    for (int h = 0; h < tot; ++h) {
      const double dx = dpdelta(px - sx[h], g.Lx);
      const double dy = dpdelta(py - sy[h], g.Ly);
      const double r2 = dx * dx + dy * dy;
      if (r2 > 0.0 && r2 < rl2) {
        const double r = sqrt(r2);
        const double prof =
            r < g.r_gran ? r / g.r_gran : 0.5 * (1.0 + cospi((r - g.r_gran) * g.inv_lane_w));
        const double s = sa[h] * prof / r;
        vx += s * dx;
        vy += s * dy;
      }
    }
  }
  if (i < g.nx && j < g.ny) {
    const size_t o = size_t(j) * g.nx + i;
    v[o] = vx;
    v[size_t(g.nx) * g.ny + o] = vy;
  }
}

__global__ void k_gran_pack(GranDev g, const double* __restrict__ v, double2* __restrict__ S) {
  const long long n = (long long)g.nx * g.ny;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    S[i] = make_double2(v[i], 0.0);
    S[n + i] = make_double2(v[n + i], 0.0);
  }
}

// divergence-free projection and the filter of eq. (3), normalised for the
// inverse transform; k = 0 and the Nyquist row and column set to zero
__global__ void k_gran_rot(GranDev g, double2* __restrict__ S) {
  const long long n = (long long)g.nx * g.ny;
  const double kN = 3.141592653589793238462643383279 / fmax(g.dx, g.dy);
  const double inv_n = 1.0 / double(n);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int iy = int(i / g.nx), ix = int(i - (long long)iy * g.nx);
    const int mx = ix < g.nx / 2 ? ix : ix - g.nx;
    const int my = iy < g.ny / 2 ? iy : iy - g.ny;
    if ((mx == 0 && my == 0) || ix == g.nx / 2 || iy == g.ny / 2) {
      S[i] = make_double2(0.0, 0.0);
      S[n + i] = make_double2(0.0, 0.0);
      continue;
    }
    const double kx = 6.283185307179586476925286766559 * mx / g.Lx;
    const double ky = 6.283185307179586476925286766559 * my / g.Ly;
    const double k2 = kx * kx + ky * ky;
    const double2 a = S[i], b = S[n + i];
    const double prx = (kx * a.x + ky * b.x) / k2, pry = (kx * a.y + ky * b.y) / k2;
    const double q = 2.0 * sqrt(k2) / kN;
    const double q2 = q * q;
    const double f = exp(-(q2 * q2)) * inv_n;
    S[i] = make_double2((a.x - kx * prx) * f, (a.y - kx * pry) * f);
    S[n + i] = make_double2((b.x - ky * prx) * f, (b.y - ky * pry) * f);
  }
}

// v_vor = v + f_rot v_rot' into out, and per-block sums of |v|^2, |v_vor|^2
// (v and out may be the same buffer: each element is read before it is
// written, by the same thread)
__global__ __launch_bounds__(256) void k_gran_combine(GranDev g, const double* v,
                                                      const double2* __restrict__ S, double* out,
                                                      double* __restrict__ part) {
  __shared__ double s1[256], s2[256];
  const long long n = (long long)g.nx * g.ny;
  double a1 = 0.0, a2 = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double vx = v[i], vy = v[n + i];
    const double wx = vx + g.f_rot * S[i].x, wy = vy + g.f_rot * S[n + i].x;
    out[i] = wx;
    out[n + i] = wy;
    a1 += vx * vx + vy * vy;
    a2 += wx * wx + wy * wy;
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1[0];
    part[kRedBlocks + blockIdx.x] = s2[0];
  }
}

// eq. (4): out *= sqrt(sum |v|^2 / sum |v_vor|^2), the partial sums added in
// a fixed order by every block
__global__ __launch_bounds__(256) void k_gran_scale(GranDev g, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double s1[256], s2[256];
  s1[threadIdx.x] = part[threadIdx.x];
  s2[threadIdx.x] = part[kRedBlocks + threadIdx.x];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  const double c = s2[0] > 0.0 ? sqrt(s1[0] / s2[0]) : 0.0;
  const long long n = 2LL * g.nx * g.ny;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] *= c;
}

GranDev dev_params(const cmhd_gran* g) {
  GranDev d;
  d.nx = g->p.nx;
  d.ny = g->p.ny;
  d.Lx = g->p.Lx;
  d.Ly = g->p.Ly;
  d.dx = g->dx;
  d.dy = g->dy;
  d.r_gran = g->p.r_gran;
  d.r_lane = g->p.r_lane;
  d.inv_lane_w = 1.0 / (g->p.r_lane - g->p.r_gran);
  d.f_rot = g->p.f_rot;
  return d;
}

bool pow2_in(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

cmhd_status cmhd_gran_create(const cmhd_gran_params* q, void* stream, cmhd_gran** out) {
  if (!q || !out) return CMHD_EINVAL;
  *out = nullptr;
  const cmhd_gran_params& p = *q;
  if (!pow2_in(p.nx) || !pow2_in(p.ny)) return CMHD_EINVAL;
  if (!(p.Lx > 0.0) || !(p.Ly > 0.0) || !std::isfinite(p.Lx) || !std::isfinite(p.Ly))
    return CMHD_EINVAL;
  if (!(p.r_gran > 0.0) || !(p.r_lane > p.r_gran) || !(p.r_excl > 0.0)) return CMHD_EINVAL;
  if (!(p.t_gran > 0.0) || !(p.v0 > 0.0) || !(p.life_var >= 0.0) || !(p.life_var < 1.0) ||
      !(p.amp_var >= 0.0) || !(p.amp_var < 1.0) || !(p.vmin_frac > 0.0) ||
      !(p.vmin_frac < 1.0 - p.amp_var) || !std::isfinite(p.f_rot))
    return CMHD_EINVAL;
  // the nearest periodic image must be unique for every granule-pixel pair
  if (!(2.0 * p.r_lane < p.Lx) || !(2.0 * p.r_lane < p.Ly)) return CMHD_EINVAL;
  const double cap = p.Lx * p.Ly / (0.8660254037844386 * p.r_excl * p.r_excl) + 16.0;
  if (!(cap < 4.0e6)) return CMHD_EINVAL;
  cmhd_gran* g = new cmhd_gran;
  g->p = p;
  g->stream = (hipStream_t)stream;
  g->dx = p.Lx / p.nx;
  g->dy = p.Ly / p.ny;
  g->capacity = int(cap);
  *out = g;
  return CMHD_OK;
}

size_t cmhd_gran_workspace_bytes(const cmhd_gran* g) {
  if (!g) return 0;
  size_t off[3];
  return gran_layout(g, off);
}

cmhd_status cmhd_gran_bind_workspace(cmhd_gran* g, void* dev_ptr, size_t bytes) {
  if (!g) return CMHD_EINVAL;
  size_t off[3];
  const size_t need = gran_layout(g, off);
  if (!dev_ptr) return gfail(g, CMHD_EINVAL, "workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0)
    return gfail(g, CMHD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need) return gfail(g, CMHD_EWORKSPACE, "workspace too small");
  g->ws = static_cast<char*>(dev_ptr);
  g->dtab = reinterpret_cast<double*>(g->ws + off[0]);
  g->spec = reinterpret_cast<double2*>(g->ws + off[1]);
  g->part = reinterpret_cast<double*>(g->ws + off[2]);
  return CMHD_OK;
}

cmhd_status cmhd_gran_update(cmhd_gran* g, double t, const double* vext, const double* unif,
                             const double* xi, long long n_pool, long long* births) {
#pragma clang fp contract(off)
  if (!g || !births || !std::isfinite(t) || n_pool < 0) return CMHD_EINVAL;
  if ((!unif || !xi) && n_pool > 0) return gfail(g, CMHD_EINVAL, "random pools are NULL");
  if (g->has_last && t < g->t_last) return gfail(g, CMHD_EINVAL, "time runs backward");
  *births = 0;
  const cmhd_gran_params& p = g->p;
  const size_t plane = size_t(p.nx) * p.ny;
  // advection of the centres
  if (vext && g->has_last) {
    const double h = t - g->t_last;
    for (size_t r = 0; r < g->tab.size(); r += kRow) {
      const double x = g->tab[r], y = g->tab[r + 1];
      const double ux = bilinear(vext, g, x, y);
      const double uy = bilinear(vext + plane, g, x, y);
      g->tab[r] = wrap(x + ux * h, p.Lx);
      g->tab[r + 1] = wrap(y + uy * h, p.Ly);
    }
  }
  // deaths: v(t) has fallen below v_min
  {
    size_t w = 0;
    for (size_t r = 0; r < g->tab.size(); r += kRow) {
      if (t > g->tab[r + 2] + 2.0 * g->tab[r + 5]) continue;
      for (int c = 0; c < kRow; ++c) g->tab[w + c] = g->tab[r + c];
      w += kRow;
    }
    g->tab.resize(w);
  }
  // free pixels of the survivors, then random sequential addition
  g->free_px.assign(plane, 1);
  for (size_t r = 0; r < g->tab.size(); r += kRow) stamp(g, g->tab[r], g->tab[r + 1], false);
  fen_build(g);
  const double vmin = p.vmin_frac * p.v0;
  long long c = 0;
  cmhd_status st = CMHD_OK;
  for (;;) {
    const int nfree = g->fen.empty() ? 0 : [&] {
      int s = 0;
      for (int idx = int(plane); idx > 0; idx -= idx & -idx) s += g->fen[idx];
      return s;
    }();
    if (nfree == 0) break;
    if (c >= n_pool) {
      st = gfail(g, CMHD_EINVAL, "random pool exhausted after " + std::to_string(c) + " births");
      break;
    }
    if (int(g->tab.size() / kRow) >= g->capacity) {
      st = gfail(g, CMHD_EINVAL, "granule table full");
      break;
    }
    long long k = (long long)std::floor(unif[c] * double(nfree));
    if (k > nfree - 1) k = nfree - 1;
    if (k < 0) k = 0;
    const int q = fen_select(g, int(k));
    const int iy = q / p.nx, ix = q - iy * p.nx;
    const double xc = double(ix) * g->dx, yc = double(iy) * g->dy;
    const double T = p.t_gran * (1.0 + p.life_var * xi[2 * c]);
    const double vmax = p.v0 * (1.0 + p.amp_var * xi[2 * c + 1]);
    const double tm = T * std::sqrt(std::fabs(std::log(vmin / vmax)));
    const double row[kRow] = {xc, yc, t, T, vmax, tm};
    g->tab.insert(g->tab.end(), row, row + kRow);
    ++c;
    stamp(g, xc, yc, true);
  }
  *births = c;
  g->has_last = true;
  g->t_last = t;
  g->dirty = true;
  return st;
}

cmhd_status cmhd_gran_velocity(cmhd_gran* g, double t, double* uh) {
  if (!g || !uh || !std::isfinite(t)) return CMHD_EINVAL;
  if (!g->ws) return gfail(g, CMHD_ESTATE, "no workspace bound");
  const GranDev d = dev_params(g);
  const int n = int(g->tab.size() / kRow);
  hipStream_t s = g->stream;
  if (g->dirty && n > 0) {
    // the table as of the last update (synchronous: the host vector may
    // change at the next update)
    hipError_t e = hipMemcpyAsync(g->dtab, g->tab.data(), g->tab.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
      return gfail(g, CMHD_EDEVICE, std::string("granule table copy: ") + hipGetErrorString(e));
  }
  g->dirty = false;
  // the render writes the granular field into the output, the combination
  // reads it back pixel by pixel before overwriting
  dim3 grid((d.nx + kTile - 1) / kTile, (d.ny + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gran_render, grid, dim3(256), 0, s, g->dtab, n, t, d, uh);
  hipLaunchKernelGGL(k_gran_pack, dim3(512), dim3(256), 0, s, d, uh, g->spec);
  KParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = d.nx;
  kp.ny = d.ny;
  kp.splane = (long long)d.nx * d.ny;
  kp.Lx = d.Lx;
  kp.Ly = d.Ly;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fft2d(kp, g->spec, 2, -1.0, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gran_rot, dim3(512), dim3(256), 0, s, d, g->spec);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = fft2d(kp, g->spec, 2, 1.0, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gran_combine, dim3(kRedBlocks), dim3(256), 0, s, d, uh, g->spec, uh,
                       g->part);
    hipLaunchKernelGGL(k_gran_scale, dim3(512), dim3(256), 0, s, d, g->part, uh);
    e = hipGetLastError();
  }
  if (e != hipSuccess)
    return gfail(g, CMHD_EDEVICE, std::string("granulation launch: ") + hipGetErrorString(e));
  return CMHD_OK;
}

cmhd_status cmhd_gran_list(const cmhd_gran* g, double* host, int cap, int* n) {
  if (!g || !n || cap < 0 || (!host && cap > 0)) return CMHD_EINVAL;
  const int m = int(g->tab.size() / kRow);
  *n = m;
  const int k = m < cap ? m : cap;
  for (int i = 0; i < k * kRow; ++i) host[i] = g->tab[i];
  return CMHD_OK;
}

const char* cmhd_gran_last_error(const cmhd_gran* g) { return g ? g->err.c_str() : "null object"; }

void cmhd_gran_destroy(cmhd_gran* g) { delete g; }

}  // extern "C"
