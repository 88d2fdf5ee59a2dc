// C ABI of the CWENO reconstruction library: mesh registration (host
// precompute + device residency) and the reconstruction launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cweno.h"
#include "dispatch.hpp"
#include "host.hpp"
#include "mesh.hpp"
#include "moving.hpp"
#include "weno.hpp"

namespace cweno_abi {

namespace {
thread_local std::string g_last_error;
std::mutex g_conf_mu;
std::vector<int> g_configured;   // devices whose kernels are configured
}  // namespace

cweno_status fail(cweno_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

cweno_status configure_device_kernels() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
  std::lock_guard<std::mutex> g(g_conf_mu);
  for (int d : g_configured)
    if (d == dev) return CWENO_OK;
  const hipError_t e = cweno::configure_all();
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel configuration failed: ") + hipGetErrorString(e));
  g_configured.push_back(dev);
  return CWENO_OK;
}

const char* last_error() { return g_last_error.c_str(); }

}  // namespace cweno_abi

using cweno_abi::DevBuf;
using cweno_abi::fail;
using cweno_abi::variant_ok;
using cweno_abi::default_variant;
using cweno_abi::make_params;
using cweno_abi::launch_block;
using cweno_abi::overlap;

namespace {

cweno_status upload(DevBuf& b, const void* src, size_t bytes, hipStream_t s, int64_t& total) {
  if (bytes == 0) return CWENO_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(CWENO_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  total += (int64_t)bytes;
  e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipMemcpyAsync failed: ") + hipGetErrorString(e));
  // pageable source: wait before the host buffer may be released
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipStreamSynchronize failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

// The classical WENO operators [row group g][entry l][Np] (g = j NE1 + k)
// uploaded in the kernel's tiled order: within each row group, the NL entries
// of a tile of cells are contiguous.  One row group at a time passes through a
// host staging buffer.
cweno_status upload_weno_tiled(DevBuf& b, const std::vector<double>& pinv, int64_t Np, int NL, hipStream_t s,
                               int64_t& total) {
  const size_t bytes = pinv.size() * sizeof(double), group = (size_t)NL * (size_t)Np;
  if (bytes == 0) return CWENO_OK;
  if (Np % cweno::kWenoTile != 0 || pinv.size() % group != 0) return fail(CWENO_E_ARG, "WENO operator size mismatch");
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(CWENO_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  total += (int64_t)bytes;
  std::vector<double> tile(group);
  constexpr int64_t T = cweno::kWenoTile;
  for (size_t g0 = 0; g0 < pinv.size(); g0 += group) {
    const double* src = pinv.data() + g0;
    cweno::parallel_for(Np / T, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t)
        for (int l = 0; l < NL; ++l)
          for (int64_t c = 0; c < T; ++c) tile[((size_t)t * NL + l) * T + c] = src[(size_t)l * Np + t * T + c];
    });
    e = hipMemcpyAsync(static_cast<double*>(b.p) + g0, tile.data(), group * sizeof(double), hipMemcpyHostToDevice, s);
    // pageable source: wait before the staging buffer is refilled
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("WENO operator upload failed: ") + hipGetErrorString(e));
  }
  return CWENO_OK;
}

cweno_status alloc_zero(DevBuf& b, size_t bytes, hipStream_t s, int64_t& total) {
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(CWENO_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  total += (int64_t)bytes;
  e = hipMemsetAsync(b.p, 0, bytes, s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipMemsetAsync failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

// Per-cell operators built on the device from the host's stencils: the
// vertices, cells and stencils go up (kept for a moving mesh,
// freed otherwise), the assembly kernel writes pinv/binv/mask in the stored
// layout, and its fault word turns into an error.
cweno_status assemble_on_device(cweno_mesh* m, const double* vertices, const int32_t* cells, int ops, hipStream_t s) {
  const int dim = m->d;
  int seg = 0, rpl = 0;
  if (!cweno::move_shape(dim, m->M, m->n_e - 1, seg, rpl, true))
    return fail(CWENO_E_ARG, "device operator assembly supports central stencils of at most 65 cells");
  int64_t scratch_bytes = 0;
  DevBuf V, C, S0, SS, SP, F;
  const std::vector<uint8_t> sp = cweno_abi::sector_rows(dim, m->nc, m->n_e, m->central, m->sectors);
  const bool keep = (m->flags & CWENO_FLAG_MOVING) != 0;
  cweno_status st;
  // frees the scratch buffers, and the mesh tables unless a moving mesh took them
  auto release = [&](bool tables) {
    for (DevBuf* b : {&V, &F})
      if (b->p) (void)hipFree(b->p);
    if (tables)
      for (DevBuf* b : {&C, &S0, &SS, &SP})
        if (b->p) (void)hipFree(b->p);
  };
  int64_t& tot = keep ? m->device_bytes : scratch_bytes;
  if ((st = upload(V, vertices, (size_t)m->n_vertices * dim * 8, s, scratch_bytes)) ||
      (st = upload(C, cells, (size_t)m->nc * (dim + 1) * 4, s, tot)) ||
      (st = upload(S0, m->central.data(), m->central.size() * 4, s, tot)) ||
      (st = upload(SS, m->sectors.data(), m->sectors.size() * 4, s, tot)) ||
      (st = upload(SP, sp.data(), sp.size(), s, tot)) || (st = alloc_zero(F, 4, s, scratch_bytes))) {
    release(true);
    return st;
  }
  const size_t Np = (size_t)m->Np, NL = (size_t)(m->nb - 1), NE1 = (size_t)(m->n_e - 1);
  const size_t nbinv = (size_t)(dim + 1) * dim * dim;
  const bool f64 = ops == CWENO_OPS_F64 || ops == CWENO_OPS_BOTH, f32 = ops == CWENO_OPS_F32 || ops == CWENO_OPS_BOTH;
  if ((f64 && ((st = alloc_zero(m->pinv64, NL * NE1 * Np * 8, s, m->device_bytes)) ||
               (st = alloc_zero(m->binv64, nbinv * Np * 8, s, m->device_bytes)))) ||
      (f32 && ((st = alloc_zero(m->pinv32, NL * NE1 * Np * 4, s, m->device_bytes)) ||
               (st = alloc_zero(m->binv32, nbinv * Np * 4, s, m->device_bytes)))) ||
      (st = alloc_zero(m->mask, Np, s, m->device_bytes))) {
    release(true);
    return st;
  }
  cweno::MParams<double> p{};
  p.V = (const double*)V.p;
  p.C = (const int32_t*)C.p;
  p.S0 = (const int32_t*)S0.p;
  p.SS = (const int32_t*)SS.p;
  p.SP = (const uint8_t*)SP.p;
  p.fault = (int*)F.p;
  p.pinv64 = (double*)m->pinv64.p;
  p.pinv32 = (float*)m->pinv32.p;
  p.binv64 = (double*)m->binv64.p;
  p.binv32 = (float*)m->binv32.p;
  p.mask = (uint8_t*)m->mask.p;
  p.Np = m->Np;
  for (int a = 0; a < 3; ++a) {
    p.box[a] = m->box[a];
    p.ibox[a] = m->box[a] != 0.0 ? 1.0 / m->box[a] : 0.0;
  }
  for (int t = 0; t < 5; ++t) p.lam[t] = m->lam[t];
  p.eps = m->eps;
  p.nc = m->nc;
  p.n_e = m->n_e;
  p.r = m->r;
  hipError_t e = cweno::launch_assemble(dim, m->M, p, seg, s);
  int fault = 0;
  std::vector<uint8_t> mask(m->nc);
  if (e == hipSuccess) e = hipMemcpyAsync(&fault, F.p, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(mask.data(), m->mask.p, m->nc, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (keep) {
    m->mvC = C;
    m->mvS0 = S0;
    m->mvSS = SS;
    m->mvSP = SP;
  }
  release(!keep);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("operator assembly failed: ") + hipGetErrorString(e));
  if (fault & 1) return fail(CWENO_E_MESH, "singular cell map (device operator assembly)");
  if (fault & 2) return fail(CWENO_E_RANK, "rank-deficient least-squares system (device operator assembly)");
  int64_t dropped = 0;
  for (int64_t i = 0; i < m->nc; ++i) dropped += (dim + 1) - __builtin_popcount(mask[i]);
  m->n_dropped = dropped;
  return CWENO_OK;
}

cweno_status upload_f32(DevBuf& b, const std::vector<double>& src, hipStream_t s, int64_t& total) {
  std::vector<float> tmp(src.size());
  for (size_t t = 0; t < src.size(); ++t) tmp[t] = (float)src[t];
  return upload(b, tmp.data(), tmp.size() * sizeof(float), s, total);
}

cweno_status check_reconstruct_args(const cweno_mesh* m, int n_vars, cweno_dtype dtype, const void* q,
                                    const void* coeffs, const void* sigma, const void* omega) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!q || !coeffs) return fail(CWENO_E_ARG, "q and coeffs must be device pointers");
  if (m->flags & CWENO_FLAG_HOST_ONLY) return fail(CWENO_E_ARG, "mesh was built host-only");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  const bool f32 = dtype == CWENO_F32;
  if ((f32 && !m->pinv32.p) || (!f32 && !m->pinv64.p))
    return fail(CWENO_E_ARG, "the mesh holds no operators of this precision");
  // averages are gathered, and the coefficients of a variable written, with 32-bit byte offsets
  if ((uint64_t)m->nc * (uint64_t)m->nb * (f32 ? 4u : 8u) >= (uint64_t(1) << 32))
    return fail(CWENO_E_ARG, "too many cells for 32-bit offsets within one variable's coefficients");
  // the kernels take every buffer as non-aliasing
  const uint64_t es = f32 ? 4 : 8, cells = (uint64_t)m->nc * (uint64_t)n_vars;
  const uint64_t nq = cells * es, nco = cells * (uint64_t)m->nb * es, nd = cells * (uint64_t)(m->d + 2) * es;
  if (overlap(q, nq, coeffs, nco) || overlap(q, nq, sigma, nd) || overlap(q, nq, omega, nd) ||
      overlap(coeffs, nco, sigma, nd) || overlap(coeffs, nco, omega, nd) || overlap(sigma, nd, omega, nd))
    return fail(CWENO_E_ARG, "q, coeffs, sigma and omega must not overlap");
  return CWENO_OK;
}

// The classical WENO scheme on a WENO mesh (FP64; no indicator or weight output).
cweno_status reconstruct_weno(const cweno_mesh* m, int n_vars, cweno_dtype dtype, const void* q, void* coeffs,
                              void* sigma, void* omega, void* hip_stream) {
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!q || !coeffs) return fail(CWENO_E_ARG, "q and coeffs must be device pointers");
  if (!m->wpinv.p) return fail(CWENO_E_ARG, "mesh was built host-only");
  if (dtype != CWENO_F64) return fail(CWENO_E_ARG, "the WENO scheme runs in FP64 only");
  if (sigma || omega) return fail(CWENO_E_ARG, "the WENO scheme reports no indicators or weights");
  const uint64_t cells = (uint64_t)m->nc * (uint64_t)n_vars;
  if (overlap(q, cells * 8u, coeffs, cells * (uint64_t)m->nb * 8u))
    return fail(CWENO_E_ARG, "q and coeffs must not overlap");
  cweno::WParams p{};
  p.q = (const double*)q;
  p.out = (double*)coeffs;
  p.pinv = (const double*)m->wpinv.p;
  p.lidx = (const uint16_t*)m->wlidx.p;
  p.halo = (const int32_t*)m->whalo.p;
  p.hoff = (const int32_t*)m->whoff.p;
  p.alive = (const uint16_t*)m->walive.p;
  p.lam0 = m->lam[0];
  p.lams = m->lam[1];
  p.eps = m->eps;
  p.nc = m->nc;
  p.Np = m->Np;
  p.NE1 = m->n_e - 1;
  p.n_s = m->n_s;
  p.r = m->r;
  // a pass takes up to kWenoMaxGroup * vbmax variables (G lanes per cell, a
  // power of two, with VB each), and no more than the LDS holds for the
  // longest block halo
  const int vbmax = cweno::weno_vb_max(m->d, m->M);
  const int lds_vars = (int)(cweno::kWenoMaxLds / ((size_t)m->wmaxH * sizeof(double)));
  const int per_pass = std::min(cweno::kWenoMaxGroup * vbmax, lds_vars);
  for (int v0 = 0; v0 < n_vars;) {
    const int n = std::min(n_vars - v0, per_pass);
    int g = 1;
    while (g * vbmax < n) g *= 2;
    const int vb = (n + g - 1) / g;
    p.v0 = v0;
    p.v1 = v0 + n;
    p.G = g;
    const hipError_t e = cweno::launch_weno(m->d, m->M, p, vb, m->wmaxH, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    v0 += n;
  }
  return CWENO_OK;
}

}  // namespace

extern "C" {

int cweno_abi_version(void) { return CWENO_ABI_VERSION; }

const char* cweno_last_error(void) { return cweno_abi::last_error(); }

const char* cweno_status_string(cweno_status st) {
  switch (st) {
    case CWENO_OK: return "ok";
    case CWENO_E_ARG: return "invalid argument";
    case CWENO_E_MESH: return "invalid mesh";
    case CWENO_E_STENCIL: return "stencil cannot be filled";
    case CWENO_E_RANK: return "rank-deficient least-squares system";
    case CWENO_E_PERIODIC: return "stencil reaches too far across the periodic box";
    case CWENO_E_NOMEM: return "out of memory";
    case CWENO_E_BUDGET: return "memory budget exceeded";
    case CWENO_E_HIP: return "HIP runtime error";
    case CWENO_E_BUSY: return "busy";
    case CWENO_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

cweno_status cweno_mesh_create(int dim, int64_t n_vertices, const double* vertices, int64_t n_cells,
                               const int32_t* cells, int degree, const cweno_options* opt,
                               void* hip_stream, cweno_mesh** out) {
  if (!out) return fail(CWENO_E_ARG, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(CWENO_E_ARG, "dim must be 2 or 3");
  if (n_vertices <= 0 || !vertices) return fail(CWENO_E_ARG, "no vertices");
  if (n_cells <= 0 || n_cells >= (int64_t(1) << 31) || !cells) return fail(CWENO_E_ARG, "bad cell count");
  if (degree < 1 || degree > 4) return fail(CWENO_E_ARG, "degree must be in 1..4");
  cweno_options o{};
  if (opt) o = *opt;
  std::unique_ptr<cweno_mesh> m;
  try {
    m.reset(new cweno_mesh());
  } catch (const std::bad_alloc&) {
    return fail(CWENO_E_NOMEM, "host allocation failed");
  }
  m->d = dim;
  m->M = degree;
  m->nb = cweno::n_basis(degree, dim);
  m->nc = n_cells;
  m->flags = o.flags;
  m->ops = o.ops;
  if (o.ops < CWENO_OPS_F64 || o.ops > CWENO_OPS_NONE) return fail(CWENO_E_ARG, "bad ops");
  if ((o.flags & CWENO_FLAG_MOVING) && (o.flags & CWENO_FLAG_HOST_ONLY))
    return fail(CWENO_E_ARG, "a moving mesh lives on the device; it cannot be host-only");
  const bool weno = (o.flags & CWENO_FLAG_WENO) != 0;
  const bool dev_ops = (o.flags & CWENO_FLAG_DEVICE_OPERATORS) != 0;
  if (dev_ops && ((o.flags & CWENO_FLAG_HOST_ONLY) || weno || o.ops == CWENO_OPS_NONE))
    return fail(CWENO_E_ARG, "device operator assembly needs a device mesh with CWENO operators");
  if (weno && (o.flags & CWENO_FLAG_MOVING)) return fail(CWENO_E_ARG, "the WENO scheme has no moving-mesh form");
  if (weno && o.ops != CWENO_OPS_F64) return fail(CWENO_E_ARG, "the WENO scheme keeps FP64 operators only");
  if (weno && (o.flags & (CWENO_FLAG_SIGMA0_POPT | CWENO_FLAG_LINEAR_WEIGHTS)))
    return fail(CWENO_E_ARG, "CWENO-only flag given for a WENO mesh");
  if (o.sector_rule != CWENO_SECTOR_CONE && o.sector_rule != CWENO_SECTOR_FACE)
    return fail(CWENO_E_ARG, "bad sector rule");
  const double f = o.stencil_factor == 0.0 ? (double)dim : o.stencil_factor;
  if (!(f > 0.0)) return fail(CWENO_E_ARG, "stencil factor must be positive");
  m->n_e = (int)std::ceil(f * m->nb);
  if (m->n_e < m->nb) return fail(CWENO_E_ARG, "central stencil smaller than the basis");
  // lam[1..] is the weight of each sectorial stencil: d+1 of them for CWENO,
  // 2(d+1) for the classical WENO scheme
  const int n_sec = (o.flags & CWENO_FLAG_WENO) ? 2 * (dim + 1) : dim + 1;
  if (o.lambda0 < 0.0) {   // the paper's pair: 1e5 for the central stencil, 1 per sector, normalised
    const double tot = 1e5 + n_sec;
    m->lam[0] = 1e5 / tot;
    for (int s = 1; s <= dim + 1; ++s) m->lam[s] = 1.0 / tot;
  } else {
    double l0 = o.lambda0 == 0.0 ? 0.95 : o.lambda0;
    if (!(l0 > 0.0 && l0 < 1.0)) return fail(CWENO_E_ARG, "lambda0 must lie in (0, 1)");
    m->lam[0] = l0;
    for (int s = 1; s <= dim + 1; ++s) m->lam[s] = (1.0 - l0) / n_sec;
  }
  m->eps = o.eps == 0.0 ? 1e-14 : o.eps;
  if (!(m->eps > 0.0)) return fail(CWENO_E_ARG, "eps must be positive");
  m->r = o.r == 0 ? 4 : o.r;
  if (m->r < 1 || m->r > 16) return fail(CWENO_E_ARG, "r must be in 1..16");
  for (int a = 0; a < 3; ++a)
    if (!(o.periodic[a] >= 0.0)) return fail(CWENO_E_ARG, "periodic box length must be >= 0");

  try {
    cweno::MeshInput in;
    in.d = dim;
    in.nv = n_vertices;
    in.V = vertices;
    in.nc = n_cells;
    in.C = cells;
    for (int a = 0; a < 3; ++a) in.box[a] = a < dim ? o.periodic[a] : 0.0;
    cweno::Geometry g;
    cweno::build_geometry(in, g);
    cweno::face_adjacency(in, m->nbr);
    cweno::Stencils st;
    cweno::build_stencils(g, m->nbr, m->n_e, o.sector_rule, st);
    if (weno) {
      cweno::WenoStencils ws;
      cweno::build_weno_stencils(g, m->nbr, st, ws);
      cweno::WenoOperators wop;
      cweno::build_weno_operators(g, ws, degree, wop);
      m->n_s = ws.n_s;
      m->weno_cells.swap(ws.cells);
      m->n_dropped = wop.n_dropped;
      // halos of the kernel's blocks over the gather lists of all stencils
      cweno::Halo wh;
      {
        cweno::Operators gl;
        gl.nc = n_cells;
        gl.Np = wop.Np;
        gl.G = m->n_s * (m->n_e - 1);
        gl.gidx.swap(wop.gidx);
        cweno::build_halo(gl, cweno::kWenoBlockCells, wh);
      }
      m->wmaxH = wh.max_len;
      if ((size_t)m->wmaxH * sizeof(double) > cweno::kWenoMaxLds)
        return fail(CWENO_E_ARG, "WENO block halo too large for LDS");
      if (!(o.flags & CWENO_FLAG_HOST_ONLY)) {
        hipStream_t s = (hipStream_t)hip_stream;
        if (hipGetDevice(&m->device) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
        cweno_status ust;
        if ((ust = upload_weno_tiled(m->wpinv, wop.pinv, wop.Np, m->nb - 1, s, m->device_bytes))) return ust;
        if ((ust = upload(m->walive, wop.alive.data(), wop.alive.size() * 2, s, m->device_bytes))) return ust;
        if ((ust = upload(m->wlidx, wh.lidx.data(), wh.lidx.size() * 2, s, m->device_bytes))) return ust;
        if ((ust = upload(m->whalo, wh.cells.data(), wh.cells.size() * 4, s, m->device_bytes))) return ust;
        if ((ust = upload(m->whoff, wh.offset.data(), wh.offset.size() * 4, s, m->device_bytes))) return ust;
      }
    } else if (dev_ops) {
      cweno::build_gather(g, st, degree, m->op);   // integer tables and Sigma; operators on the device
    } else if (o.ops != CWENO_OPS_NONE) {
      cweno::build_operators(g, st, degree, m->op);
    }
    m->central.swap(st.central);
    m->sectors.swap(st.sectors);
  } catch (const cweno::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(CWENO_E_NOMEM, "host allocation failed during precompute");
  } catch (const std::exception& e) {
    return fail(CWENO_E_ARG, e.what());
  }
  if (o.ops == CWENO_OPS_NONE || weno) {   // no stored CWENO operators
    m->op.d = dim;
    m->op.M = degree;
    m->op.nb = m->nb;
    m->op.n_e = m->n_e;
    m->op.nc = n_cells;
    m->op.Np = (n_cells + 63) / 64 * 64;
    cweno::sigma_matrix(dim, degree, m->op.sigma);
  }
  m->G = m->op.G;
  m->Np = m->op.Np;
  for (int a = 0; a < 3; ++a) m->box[a] = a < dim ? o.periodic[a] : 0.0;
  m->n_vertices = n_vertices;
  // the kernels address each block of operator or index rows with 32-bit byte offsets
  {
    const uint64_t Np = (uint64_t)m->Np, lim = uint64_t(1) << 32;
    if ((uint64_t)(m->nb - 1) * Np * 8u >= lim || (uint64_t)(dim + 1) * dim * dim * Np * 8u >= lim ||
        (uint64_t)(m->G + 1) * Np * 4u >= lim)
      return fail(CWENO_E_ARG, "mesh too large for 32-bit offsets within an operator block (split it)");
  }
  if (!weno && !dev_ops) m->n_dropped = m->op.n_dropped;

  if (!(o.flags & CWENO_FLAG_HOST_ONLY) && !weno) {
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipGetDevice(&m->device) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
    if (cweno_status cst = cweno_abi::configure_device_kernels()) return cst;
    const cweno::Operators& op = m->op;
    cweno_status st;
    if (dev_ops) {
      try {
        if ((st = assemble_on_device(m.get(), vertices, cells, o.ops, s))) return st;
      } catch (const std::bad_alloc&) {
        return fail(CWENO_E_NOMEM, "host allocation failed during device assembly");
      }
    } else if (o.flags & CWENO_FLAG_MOVING) {
      // connectivity and stencils for the moving-mesh kernel
      if ((st = upload(m->mvC, cells, (size_t)n_cells * (dim + 1) * 4, s, m->device_bytes))) return st;
      if ((st = upload(m->mvS0, m->central.data(), m->central.size() * 4, s, m->device_bytes))) return st;
      if ((st = upload(m->mvSS, m->sectors.data(), m->sectors.size() * 4, s, m->device_bytes))) return st;
      const std::vector<uint8_t> sp = cweno_abi::sector_rows(dim, n_cells, m->n_e, m->central, m->sectors);
      if ((st = upload(m->mvSP, sp.data(), sp.size(), s, m->device_bytes))) return st;
    }
    if (o.ops == CWENO_OPS_F64 || o.ops == CWENO_OPS_BOTH) {
      if (!dev_ops) {
        if ((st = upload(m->pinv64, op.pinv.data(), op.pinv.size() * 8, s, m->device_bytes))) return st;
        if ((st = upload(m->binv64, op.binv.data(), op.binv.size() * 8, s, m->device_bytes))) return st;
      }
      if ((st = upload(m->sigma64, op.sigma.data(), op.sigma.size() * 8, s, m->device_bytes))) return st;
    }
    if (o.ops == CWENO_OPS_F32 || o.ops == CWENO_OPS_BOTH) {
      if (!dev_ops) {
        if ((st = upload_f32(m->pinv32, op.pinv, s, m->device_bytes))) return st;
        if ((st = upload_f32(m->binv32, op.binv, s, m->device_bytes))) return st;
      }
      if ((st = upload_f32(m->sigma32, op.sigma, s, m->device_bytes))) return st;
    }
    if (o.ops != CWENO_OPS_NONE) {
      if ((st = upload(m->gidx, op.gidx.data(), op.gidx.size() * 4, s, m->device_bytes))) return st;
      if ((st = upload(m->secpos, op.secpos.data(), op.secpos.size(), s, m->device_bytes))) return st;
      if (!dev_ops && (st = upload(m->mask, op.mask.data(), op.mask.size(), s, m->device_bytes))) return st;
      try {
        cweno::Halo h;
        cweno::build_halo(op, cweno::kHaloBlock, h);
        if ((st = upload(m->halo, h.cells.data(), h.cells.size() * 4, s, m->device_bytes))) return st;
        if ((st = upload(m->hoff, h.offset.data(), h.offset.size() * 4, s, m->device_bytes))) return st;
        if ((st = upload(m->lidx, h.lidx.data(), h.lidx.size() * 2, s, m->device_bytes))) return st;
        m->maxH = h.max_len;
      } catch (const cweno::Error&) {
        m->maxH = 0;   // halos too large: the halo kernel is not used for this mesh
      }
    }
    // the device holds the operators now; keep only what the host-side dumps need
    std::vector<double>().swap(m->op.pinv);
    std::vector<double>().swap(m->op.binv);
    std::vector<int32_t>().swap(m->op.gidx);
    std::vector<uint8_t>().swap(m->op.secpos);
  }
  for (int t = 0; t < 2; ++t)
    for (int vb = 0; vb < 10; ++vb) m->variant[t][vb] = vb == 0 ? -1 : default_variant(m.get(), vb, t == 1);
  *out = m.release();
  return CWENO_OK;
}

cweno_status cweno_mesh_destroy(cweno_mesh* mesh) {
  delete mesh;
  return CWENO_OK;
}

cweno_status cweno_mesh_info(const cweno_mesh* m, int64_t* n_cells, int* n_basis, int* n_e, int* gather_len,
                             int64_t* device_bytes, int64_t* n_dropped) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (n_cells) *n_cells = m->nc;
  if (n_basis) *n_basis = m->nb;
  if (n_e) *n_e = m->n_e;
  if (gather_len) *gather_len = m->G;
  if (device_bytes) *device_bytes = m->device_bytes;
  if (n_dropped) *n_dropped = m->n_dropped;
  return CWENO_OK;
}

cweno_status cweno_mesh_tables(const cweno_mesh* m, int32_t* face_nbr, int32_t* stencil, int32_t* sectors) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (face_nbr) std::memcpy(face_nbr, m->nbr.data(), m->nbr.size() * 4);
  if (stencil) std::memcpy(stencil, m->central.data(), m->central.size() * 4);
  if (sectors) std::memcpy(sectors, m->sectors.data(), m->sectors.size() * 4);
  return CWENO_OK;
}

cweno_status cweno_mesh_weno_tables(const cweno_mesh* m, int* n_stencils, int32_t* stencils) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (m->n_s == 0) return fail(CWENO_E_ARG, "not a WENO mesh");
  if (n_stencils) *n_stencils = m->n_s;
  if (stencils) std::memcpy(stencils, m->weno_cells.data(), m->weno_cells.size() * 4);
  return CWENO_OK;
}

cweno_status cweno_mesh_operators(const cweno_mesh* m, int64_t cell, double* pinv, double* binv, double* sigma) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (cell < 0 || cell >= m->nc) return fail(CWENO_E_ARG, "cell out of range");
  const cweno::Operators& op = m->op;
  const size_t Np = (size_t)m->Np;
  if ((pinv || binv) && op.pinv.empty())
    return fail(CWENO_E_ARG, "per-cell operators are kept on the host only for host-only meshes");
  const int NE1 = m->n_e - 1, NL = m->nb - 1, d = m->d;
  if (pinv)
    for (int l = 0; l < NL; ++l)
      for (int k = 0; k < NE1; ++k) pinv[l * NE1 + k] = op.pinv[((size_t)k * NL + l) * Np + cell];
  if (binv)
    for (int t = 0; t < (d + 1) * d * d; ++t) binv[t] = op.binv[(size_t)t * Np + cell];
  if (sigma) std::memcpy(sigma, op.sigma.data(), op.sigma.size() * 8);
  return CWENO_OK;
}

cweno_status cweno_reconstruct(const cweno_mesh* m, int n_vars, cweno_dtype dtype, const void* q, void* coeffs,
                               void* sigma, void* omega, void* hip_stream) {
  if (m && m->n_s > 0) return reconstruct_weno(m, n_vars, dtype, q, coeffs, sigma, omega, hip_stream);
  cweno_status st = check_reconstruct_args(m, n_vars, dtype, q, coeffs, sigma, omega);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const bool f32 = dtype == CWENO_F32;
  for (int v0 = 0; v0 < n_vars;) {
    const int vb = cweno_abi::pick_vb_mesh(m, n_vars - v0, f32);
    const int k = m->variant[f32][vb];
    hipError_t e = launch_block(m, f32, q, coeffs, sigma, omega, v0, vb, k, s);
    if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    v0 += vb;
  }
  return CWENO_OK;
}

cweno_status cweno_mesh_set_variant(cweno_mesh* m, cweno_dtype dtype, int vb, int variant) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  if (vb < 1 || vb > 9) return fail(CWENO_E_ARG, "variable block out of range");
  if (variant < 0 || variant >= cweno::kNumVariants) return fail(CWENO_E_ARG, "variant out of range");
  if (!variant_ok(m, vb, variant, dtype == CWENO_F32))
    return fail(CWENO_E_ARG, "variant not instantiated for this block");
  m->variant[dtype == CWENO_F32][vb] = variant;
  return CWENO_OK;
}

cweno_status cweno_mesh_get_variant(const cweno_mesh* m, cweno_dtype dtype, int vb, int* variant, int* kind,
                                    int* kc) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  if (vb < 1 || vb > 9) return fail(CWENO_E_ARG, "variable block out of range");
  const int k = m->variant[dtype == CWENO_F32][vb];
  if (variant) *variant = k;
  if (kind) *kind = k >= 0 ? cweno::kVariants[k].kind : -1;
  if (kc) *kc = k >= 0 ? cweno::kVariants[k].kc : 0;
  return CWENO_OK;
}

int cweno_num_variants(void) { return cweno::kNumVariants; }

cweno_status cweno_mesh_tune(cweno_mesh* m, int n_vars, cweno_dtype dtype, const void* q, void* coeffs,
                             int repeats, void* hip_stream, double* best_ms) {
  cweno_status st = check_reconstruct_args(m, n_vars, dtype, q, coeffs, nullptr, nullptr);
  if (st) return st;
  if (repeats < 1) return fail(CWENO_E_ARG, "repeats must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  const bool f32 = dtype == CWENO_F32;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(CWENO_E_HIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CWENO_E_HIP, "hipEventCreate failed");
  }
  double total = 0.0;
  st = CWENO_OK;
  for (int v0 = 0; v0 < n_vars && st == CWENO_OK;) {
    const int vb = cweno_abi::pick_vb_mesh(m, n_vars - v0, f32);
    float best = 0.0f;
    int best_k = -1;
    for (int k = 0; k < cweno::kNumVariants && st == CWENO_OK; ++k) {
      if (!variant_ok(m, vb, k, f32)) continue;
      hipError_t e = launch_block(m, f32, q, coeffs, nullptr, nullptr, v0, vb, k, s);   // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int t = 0; t < repeats && e == hipSuccess; ++t)
        e = launch_block(m, f32, q, coeffs, nullptr, nullptr, v0, vb, k, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = fail(CWENO_E_HIP, std::string("tuning launch failed: ") + hipGetErrorString(e));
        break;
      }
      if (best_k < 0 || ms < best) { best = ms; best_k = k; }
    }
    if (st == CWENO_OK) {
      m->variant[f32][vb] = best_k;
      total += best / repeats;
    }
    v0 += vb;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == CWENO_OK && best_ms) *best_ms = total;
  return st;
}

}  // extern "C"
