// C ABI of the moving-mesh reconstruction (operators rebuilt per call).
#include <hip/hip_runtime.h>

#include <string>

#include "cweno.h"
#include "mesh.hpp"
#include "moving.hpp"

using cweno_abi::fail;
using cweno_abi::overlap;

namespace {

template <typename T>
cweno::MParams<T> moving_params(const cweno_mesh* m, const double* vertices, int n_vars, const void* q,
                                void* coeffs, void* sigma, void* omega, int* fault) {
  cweno::MParams<T> p{};
  p.V = vertices;
  p.C = (const int32_t*)m->mvC.p;
  p.S0 = (const int32_t*)m->mvS0.p;
  p.SS = (const int32_t*)m->mvSS.p;
  p.SP = (const uint8_t*)m->mvSP.p;
  p.q = (const T*)q;
  p.out = (T*)coeffs;
  p.sig = (T*)sigma;
  p.om = (T*)omega;
  p.fault = fault;
  for (int a = 0; a < 3; ++a) {
    p.box[a] = m->box[a];
    p.ibox[a] = m->box[a] != 0.0 ? 1.0 / m->box[a] : 0.0;
  }
  for (int s = 0; s < 5; ++s) p.lam[s] = m->lam[s];
  p.eps = m->eps;
  p.nc = m->nc;
  p.n_e = m->n_e;
  p.nv = n_vars;
  p.r = m->r;
  p.sigma0_popt = (m->flags & CWENO_FLAG_SIGMA0_POPT) ? 1 : 0;
  p.linear_w = (m->flags & CWENO_FLAG_LINEAR_WEIGHTS) ? 1 : 0;
  return p;
}

}  // namespace

extern "C" cweno_status cweno_reconstruct_moving(const cweno_mesh* m, const double* vertices, int n_vars,
                                                 cweno_dtype dtype, const void* q, void* coeffs, void* sigma,
                                                 void* omega, int* fault, void* hip_stream) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (!m->mvC.p) return fail(CWENO_E_ARG, "mesh was not created with CWENO_FLAG_MOVING");
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!vertices || !q || !coeffs) return fail(CWENO_E_ARG, "vertices, q and coeffs must be device pointers");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  const bool f32 = dtype == CWENO_F32;
  int seg = m->mv_seg, rpl = m->mv_rpl;
  if (seg == 0 && !cweno::move_shape(m->d, m->M, m->n_e - 1, seg, rpl))
    return fail(CWENO_E_ARG, "central stencil too large for the moving-mesh kernel");
  const uint64_t es = f32 ? 4 : 8, cells = (uint64_t)m->nc * (uint64_t)n_vars;
  const uint64_t nq = cells * es, nco = cells * (uint64_t)m->nb * es, nd = cells * (uint64_t)(m->d + 2) * es;
  const uint64_t nvx = (uint64_t)m->n_vertices * (uint64_t)m->d * 8u;
  const void* bufs[6] = {vertices, q, coeffs, sigma, omega, fault};
  const uint64_t lens[6] = {nvx, nq, nco, nd, nd, fault ? 4u : 0u};
  for (int a = 0; a < 6; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (overlap(bufs[a], lens[a], bufs[b], lens[b]))
        return fail(CWENO_E_ARG, "vertices, q, coeffs, sigma, omega and fault must not overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e;
  if (f32)
    e = cweno::launch_moving(m->d, m->M, moving_params<float>(m, vertices, n_vars, q, coeffs, sigma, omega, fault),
                             seg, rpl, s);
  else
    e = cweno::launch_moving(m->d, m->M, moving_params<double>(m, vertices, n_vars, q, coeffs, sigma, omega, fault),
                             seg, rpl, s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

extern "C" cweno_status cweno_mesh_set_moving_shape(cweno_mesh* m, int seg, int rpl) {
  if (!m) return fail(CWENO_E_ARG, "mesh is NULL");
  if (!m->mvC.p) return fail(CWENO_E_ARG, "mesh was not created with CWENO_FLAG_MOVING");
  if (seg == 0 && rpl == 0) {
    m->mv_seg = m->mv_rpl = 0;
    return CWENO_OK;
  }
  if (!cweno::move_shape_ok(m->d, m->M, seg, rpl))
    return fail(CWENO_E_ARG, "segment shape not instantiated for this dimension and degree");
  if (m->n_e - 1 > seg * rpl) return fail(CWENO_E_ARG, "segment shape too small for the central stencil");
  m->mv_seg = seg;
  m->mv_rpl = rpl;
  return CWENO_OK;
}

extern "C" cweno_status cweno_mesh_moving_shape(const cweno_mesh* m, int* seg, int* rpl) {
  if (!m || !seg || !rpl) return fail(CWENO_E_ARG, "NULL argument");
  if (!m->mvC.p) return fail(CWENO_E_ARG, "mesh was not created with CWENO_FLAG_MOVING");
  int s = m->mv_seg, r = m->mv_rpl;
  if (s == 0 && !cweno::move_shape(m->d, m->M, m->n_e - 1, s, r))
    return fail(CWENO_E_ARG, "central stencil too large for the moving-mesh kernel");
  *seg = s;
  *rpl = r;
  return CWENO_OK;
}
