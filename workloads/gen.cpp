// Seeded synthetic workloads for hybrid-voxel-format ray tracing.
//
// This module produces INPUTS only: occupancy sets (as strictly ascending Morton codes)
// and ray arrays. It holds none of the traversal arithmetic. Both the CPU oracle and the
// GPU library consume what it produces; neither links it.
//
// Random numbers: counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): the 64-bit finalizer applied to
// seed-derived counters, so every draw is a pure function of (seed, stream, index).
//
// Scenes: unions of spheres and tori given by exact signed distance functions (SDFs),
// taken either as solids (sdf <= 0) or as 1-voxel shells (sdf <= 0 and some
// 6-neighbour has sdf > 0). Shells are found by recursive subdivision with
// Lipschitz-1 culling, which skips blocks that provably contain no shell voxel.
//
// Morton order: x is bit 0, y bit 1, z bit 2 of each 3-bit group (the paper's Morton
// figure orders a 2-D grid x-first, then y).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t rng_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t key = mix64(seed + 0x9E3779B97F4A7C15ull * (stream + 1));
  return mix64(key + 0x9E3779B97F4A7C15ull * (idx + 1));
}
inline double rng_unit(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(rng_u64(seed, stream, idx) >> 11) * 0x1.0p-53;
}
inline double rng_range(uint64_t seed, uint64_t stream, uint64_t idx, double a, double b) {
  return a + (b - a) * rng_unit(seed, stream, idx);
}

inline uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
  v = (v ^ (v >> 32)) & 0x1FFFFFull;
  return v;
}
inline uint64_t morton_enc(uint64_t x, uint64_t y, uint64_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Stream ids (keep stable: changing them changes every workload).
enum : uint64_t {
  ST_SPH_C = 1, ST_SPH_R = 2, ST_TOR_C = 3, ST_TOR_RR = 4, ST_TOR_AX = 5, ST_NOISE = 6,
  ST_CAM = 7, ST_RAY_O = 8, ST_RAY_D = 9, ST_BOUNCE = 10, ST_BERN = 11
};

struct Prim {
  int type;        // 0 sphere, 1 torus
  double c[3];     // centre
  double ax[3];    // torus axis (unit)
  double R, r;     // sphere radius in R; torus major R, minor r
};

inline double prim_sdf(const Prim& p, double x, double y, double z) {
  double qx = x - p.c[0], qy = y - p.c[1], qz = z - p.c[2];
  double q2 = qx * qx + qy * qy + qz * qz;
  if (p.type == 0) return std::sqrt(q2) - p.R;
  double h = qx * p.ax[0] + qy * p.ax[1] + qz * p.ax[2];
  double rad2 = q2 - h * h;
  double rad = rad2 > 0.0 ? std::sqrt(rad2) : 0.0;
  double a = rad - p.R;
  return std::sqrt(a * a + h * h) - p.r;
}

struct Result {
  std::vector<uint64_t> codes;
};

// Shell generator state.
struct ShellGen {
  std::vector<Prim> prims;
  int64_t N;
  static constexpr int LEAF = 4;

  double sdf_min(const int* cand, int nc, double x, double y, double z) const {
    double m = INFINITY;
    for (int i = 0; i < nc; ++i) m = std::min(m, prim_sdf(prims[cand[i]], x, y, z));
    return m;
  }

  void recurse(int64_t lx, int64_t ly, int64_t lz, int64_t s, const std::vector<int>& cand,
               std::vector<uint64_t>& out) const {
    double cx = lx + 0.5 * s, cy = ly + 0.5 * s, cz = lz + 0.5 * s;
    // Radius (in voxel units) covering every voxel centre of the block and its 6-neighbours.
    double R = std::sqrt(3.0) * 0.5 * (double)(s - 1) + 1.0 + 1e-7;
    std::vector<double> dv(cand.size());
    double m = INFINITY;
    for (size_t i = 0; i < cand.size(); ++i) {
      dv[i] = prim_sdf(prims[cand[i]], cx, cy, cz);
      m = std::min(m, dv[i]);
    }
    if (m > R || m < -R) return;  // Lipschitz-1: one sign over the block and its neighbours
    std::vector<int> nc;
    nc.reserve(cand.size());
    for (size_t i = 0; i < cand.size(); ++i)
      if (dv[i] <= m + 2.0 * R) nc.push_back(cand[i]);
    if (s <= LEAF) {
      int64_t cells = s * s * s;
      for (int64_t k = 0; k < cells; ++k) {
        int64_t x = lx + (int64_t)compact3((uint64_t)k), y = ly + (int64_t)compact3((uint64_t)k >> 1),
                z = lz + (int64_t)compact3((uint64_t)k >> 2);
        double px = x + 0.5, py = y + 0.5, pz = z + 0.5;
        if (sdf_min(nc.data(), (int)nc.size(), px, py, pz) > 0.0) continue;
        bool shell = sdf_min(nc.data(), (int)nc.size(), px - 1, py, pz) > 0.0 ||
                     sdf_min(nc.data(), (int)nc.size(), px + 1, py, pz) > 0.0 ||
                     sdf_min(nc.data(), (int)nc.size(), px, py - 1, pz) > 0.0 ||
                     sdf_min(nc.data(), (int)nc.size(), px, py + 1, pz) > 0.0 ||
                     sdf_min(nc.data(), (int)nc.size(), px, py, pz - 1) > 0.0 ||
                     sdf_min(nc.data(), (int)nc.size(), px, py, pz + 1) > 0.0;
        if (shell) out.push_back(morton_enc((uint64_t)x, (uint64_t)y, (uint64_t)z));
      }
      return;
    }
    int64_t h = s / 2;
    for (int o = 0; o < 8; ++o)
      recurse(lx + (o & 1) * h, ly + ((o >> 1) & 1) * h, lz + ((o >> 2) & 1) * h, h, nc, out);
  }
};

void make_prims(uint64_t seed, int64_t N, int n_sph, int n_tor, double scale, std::vector<Prim>& prims) {
  for (int i = 0; i < n_sph; ++i) {
    Prim p{};
    p.type = 0;
    for (int a = 0; a < 3; ++a) p.c[a] = rng_range(seed, ST_SPH_C, 3 * i + a, 0.15 * N, 0.85 * N);
    p.R = rng_range(seed, ST_SPH_R, i, 0.04 * N * scale, 0.12 * N * scale);
    prims.push_back(p);
  }
  for (int i = 0; i < n_tor; ++i) {
    Prim p{};
    p.type = 1;
    for (int a = 0; a < 3; ++a) p.c[a] = rng_range(seed, ST_TOR_C, 3 * i + a, 0.15 * N, 0.85 * N);
    p.R = rng_range(seed, ST_TOR_RR, 2 * i, 0.05 * N * scale, 0.12 * N * scale);
    p.r = rng_range(seed, ST_TOR_RR, 2 * i + 1, 0.01 * N * scale, 0.03 * N * scale);
    double zc = rng_range(seed, ST_TOR_AX, 2 * i, -1.0, 1.0);
    double ph = rng_range(seed, ST_TOR_AX, 2 * i + 1, 0.0, 2.0 * M_PI);
    double sr = std::sqrt(std::max(0.0, 1.0 - zc * zc));
    p.ax[0] = sr * std::cos(ph);
    p.ax[1] = sr * std::sin(ph);
    p.ax[2] = zc;
    prims.push_back(p);
  }
}

struct Ray {
  float ox, oy, oz, tmin, dx, dy, dz, tmax;
};
struct Hit {
  int32_t x, y, z;
  float t;
};

}  // namespace

extern "C" {

uint64_t wl_morton_encode(uint32_t x, uint32_t y, uint32_t z) { return morton_enc(x, y, z); }
void wl_morton_decode(uint64_t c, uint32_t* x, uint32_t* y, uint32_t* z) {
  *x = (uint32_t)compact3(c);
  *y = (uint32_t)compact3(c >> 1);
  *z = (uint32_t)compact3(c >> 2);
}
void wl_morton_encode_many(const int32_t* xyz, int64_t n, uint64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = morton_enc(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
}
void wl_morton_decode_many(const uint64_t* c, int64_t n, int32_t* xyz) {
  for (int64_t i = 0; i < n; ++i) {
    xyz[3 * i] = (int32_t)compact3(c[i]);
    xyz[3 * i + 1] = (int32_t)compact3(c[i] >> 1);
    xyz[3 * i + 2] = (int32_t)compact3(c[i] >> 2);
  }
}

uint64_t wl_rng_u64(uint64_t seed, uint64_t stream, uint64_t idx) { return rng_u64(seed, stream, idx); }

// Result handles for variable-length code lists.
void* wl_result_new() { return new Result(); }
int64_t wl_result_size(void* h) { return (int64_t)((Result*)h)->codes.size(); }
void wl_result_copy(void* h, uint64_t* out) {
  auto& v = ((Result*)h)->codes;
  if (!v.empty()) std::memcpy(out, v.data(), v.size() * 8);
}
void wl_result_free(void* h) { delete (Result*)h; }

// Shell of a union of n_sph spheres and n_tor tori in an N^3 grid (N = 2^log2n).
// scale multiplies every radius range. Returns a handle holding ascending Morton codes.
void* wl_scene_shell(uint64_t seed, int log2n, int n_sph, int n_tor, double scale, int nthreads) {
  ShellGen g;
  g.N = (int64_t)1 << log2n;
  make_prims(seed, g.N, n_sph, n_tor, scale, g.prims);
  std::vector<int> all(g.prims.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
  // Split the grid into 8^k Morton-ordered top blocks; each thread fills whole blocks.
  int split = 0;
  while (split < 3 && ((int64_t)1 << (log2n - split - 1)) >= ShellGen::LEAF) ++split;
  int64_t nb = (int64_t)1 << (3 * split);
  int64_t bs = g.N >> split;
  std::vector<std::vector<uint64_t>> parts(nb);
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (;;) {
      int64_t b = next.fetch_add(1);
      if (b >= nb) break;
      int64_t lx = (int64_t)compact3((uint64_t)b) * bs, ly = (int64_t)compact3((uint64_t)b >> 1) * bs,
              lz = (int64_t)compact3((uint64_t)b >> 2) * bs;
      g.recurse(lx, ly, lz, bs, all, parts[b]);
    }
  };
  int nt = std::max(1, nthreads);
  std::vector<std::thread> th;
  for (int i = 0; i < nt - 1; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  auto* res = new Result();
  size_t tot = 0;
  for (auto& p : parts) tot += p.size();
  res->codes.reserve(tot);
  for (auto& p : parts) res->codes.insert(res->codes.end(), p.begin(), p.end());
  return res;
}

// Solid union of n_sph spheres (centres U[N/4, 3N/4]^3, radii U[rmin, rmax] * N/64),
// OR-ed with i.i.d. Bernoulli(noise) voxels, over an N^3 grid visited in Morton order.
void* wl_scene_solid_noise(uint64_t seed, int log2n, int n_sph, double rmin, double rmax, double noise) {
  int64_t N = (int64_t)1 << log2n;
  std::vector<Prim> prims;
  for (int i = 0; i < n_sph; ++i) {
    Prim p{};
    p.type = 0;
    for (int a = 0; a < 3; ++a) p.c[a] = rng_range(seed, ST_SPH_C, 3 * i + a, 0.25 * N, 0.75 * N);
    p.R = rng_range(seed, ST_SPH_R, i, rmin, rmax) * (double)N / 64.0;
    prims.push_back(p);
  }
  auto* res = new Result();
  uint64_t total = (uint64_t)1 << (3 * log2n);
  for (uint64_t c = 0; c < total; ++c) {
    double x = compact3(c) + 0.5, y = compact3(c >> 1) + 0.5, z = compact3(c >> 2) + 0.5;
    bool occ = rng_unit(seed, ST_NOISE, c) < noise;
    for (size_t i = 0; i < prims.size() && !occ; ++i) occ = prim_sdf(prims[i], x, y, z) <= 0.0;
    if (occ) res->codes.push_back(c);
  }
  return res;
}

// i.i.d. Bernoulli(p) occupancy over a 2^ex x 2^ey x 2^ez grid (Morton codes of the
// in-bounds voxels, ascending). For small test volumes.
void* wl_scene_bernoulli(uint64_t seed, int ex, int ey, int ez, double p) {
  int m = std::max(ex, std::max(ey, ez));
  uint64_t total = (uint64_t)1 << (3 * m);
  auto* res = new Result();
  for (uint64_t c = 0; c < total; ++c) {
    uint64_t x = compact3(c), y = compact3(c >> 1), z = compact3(c >> 2);
    if (x >> ex || y >> ey || z >> ez) continue;
    if (rng_unit(seed, ST_BERN, c) < p) res->codes.push_back(c);
  }
  return res;
}

// Pinhole camera on a seeded orbit about the grid centre. Orbit radius U[rmin, rmax]
// times the largest extent, azimuth U[0, 2pi), elevation U[-60, 60] degrees, up = +z,
// vertical field of view fov_deg. Rays through pixel centres, row-major; directions
// computed in double, normalised, rounded to fp32. tmin = 0, tmax = +inf.
void wl_camera_rays(uint64_t seed, uint64_t view, int nx, int ny, int nz, int W, int H, double fov_deg,
                    double rmin, double rmax, Ray* out) {
  double N = std::max(nx, std::max(ny, nz));
  double cen[3] = {0.5 * nx, 0.5 * ny, 0.5 * nz};
  double rad = rng_range(seed, ST_CAM, 4 * view, rmin, rmax) * N;
  double az = rng_range(seed, ST_CAM, 4 * view + 1, 0.0, 2.0 * M_PI);
  double el = rng_range(seed, ST_CAM, 4 * view + 2, -M_PI / 3.0, M_PI / 3.0);
  double eye[3] = {cen[0] + rad * std::cos(el) * std::cos(az), cen[1] + rad * std::cos(el) * std::sin(az),
                   cen[2] + rad * std::sin(el)};
  double f[3] = {cen[0] - eye[0], cen[1] - eye[1], cen[2] - eye[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double& v : f) v /= fl;
  double up[3] = {0, 0, 1};
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double& v : r) v /= rl;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  double th = std::tan(0.5 * fov_deg * M_PI / 180.0);
  double aspect = (double)W / (double)H;
  for (int j = 0; j < H; ++j)
    for (int i = 0; i < W; ++i) {
      double sx = (2.0 * (i + 0.5) / W - 1.0) * th * aspect;
      double sy = (1.0 - 2.0 * (j + 0.5) / H) * th;
      double d[3];
      for (int a = 0; a < 3; ++a) d[a] = f[a] + sx * r[a] + sy * u[a];
      double dl = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      Ray& ry = out[(int64_t)j * W + i];
      ry.ox = (float)eye[0];
      ry.oy = (float)eye[1];
      ry.oz = (float)eye[2];
      ry.dx = (float)(d[0] / dl);
      ry.dy = (float)(d[1] / dl);
      ry.dz = (float)(d[2] / dl);
      ry.tmin = 0.0f;
      ry.tmax = INFINITY;
    }
}

// n rays with origins uniform in the grid's bounding box and directions uniform on the
// unit sphere. tmin = 0, tmax = +inf.
void wl_random_rays(uint64_t seed, int nx, int ny, int nz, int64_t n, Ray* out) {
  for (int64_t i = 0; i < n; ++i) {
    double o[3] = {rng_range(seed, ST_RAY_O, 3 * i, 0.0, nx), rng_range(seed, ST_RAY_O, 3 * i + 1, 0.0, ny),
                   rng_range(seed, ST_RAY_O, 3 * i + 2, 0.0, nz)};
    double zc = rng_range(seed, ST_RAY_D, 2 * i, -1.0, 1.0);
    double ph = rng_range(seed, ST_RAY_D, 2 * i + 1, 0.0, 2.0 * M_PI);
    double sr = std::sqrt(std::max(0.0, 1.0 - zc * zc));
    Ray& r = out[i];
    r.ox = (float)o[0];
    r.oy = (float)o[1];
    r.oz = (float)o[2];
    r.dx = (float)(sr * std::cos(ph));
    r.dy = (float)(sr * std::sin(ph));
    r.dz = (float)zc;
    r.tmin = 0.0f;
    r.tmax = INFINITY;
  }
}

// One cosine-weighted hemisphere bounce ray per primary hit. The surface normal is the
// outward normal of the hit voxel's entry face, found in double precision as the face
// whose plane the ray crosses last; a ray that starts inside its hit voxel gets no
// bounce. Origin = hit point + 2^-6 * normal (double, rounded to fp32); direction is
// cosine-weighted about the normal; tmin = 0, tmax = +inf. Writes the bounce rays
// compactly and, in src[], the primary index each came from. Returns the count.
int64_t wl_bounce_rays(uint64_t seed, const Ray* rays, const Hit* hits, int64_t n, Ray* out, int64_t* src) {
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    const Hit& h = hits[i];
    if (h.x < 0) continue;
    const Ray& r = rays[i];
    double o[3] = {r.ox, r.oy, r.oz}, d[3] = {r.dx, r.dy, r.dz};
    int v[3] = {h.x, h.y, h.z};
    int best = -1;
    double bt = -INFINITY;
    for (int a = 0; a < 3; ++a) {
      if (d[a] == 0.0) continue;
      double plane = v[a] + (d[a] < 0 ? 1.0 : 0.0);
      double tp = (plane - o[a]) / d[a];
      if (tp > bt) {
        bt = tp;
        best = a;
      }
    }
    if (best < 0 || !(bt > (double)r.tmin)) continue;
    double nrm[3] = {0, 0, 0};
    nrm[best] = d[best] > 0 ? -1.0 : 1.0;
    double t = h.t;
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + t * d[a] + 0x1.0p-6 * nrm[a];
    // Orthonormal frame about the normal.
    double ta[3] = {0, 0, 0}, tb[3] = {0, 0, 0};
    ta[(best + 1) % 3] = 1.0;
    tb[(best + 2) % 3] = 1.0;
    double u1 = rng_unit(seed, ST_BOUNCE, 2 * i), u2 = rng_unit(seed, ST_BOUNCE, 2 * i + 1);
    double rr = std::sqrt(u1), phi = 2.0 * M_PI * u2;
    double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(std::max(0.0, 1.0 - u1));
    double dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = lx * ta[a] + ly * tb[a] + lz * nrm[a];
    Ray& q = out[m];
    q.ox = (float)p[0];
    q.oy = (float)p[1];
    q.oz = (float)p[2];
    q.dx = (float)dd[0];
    q.dy = (float)dd[1];
    q.dz = (float)dd[2];
    q.tmin = 0.0f;
    q.tmax = INFINITY;
    src[m] = i;
    ++m;
  }
  return m;
}

}  // extern "C"
