// Point values of the reconstruction polynomials (the step after the
// reconstruction: the predictor and the fluxes consume the reconstruction at
// quadrature points of each cell, Sec. 2.2-2.3).
//
// A point set is a list of reference coordinates, the same for every cell
// (each cell's coefficients live in its own reference frame, so a reference
// point is the same relative place in every cell).  Its basis matrix
// phi[q][l] = psi_l(xi_q) is built once on the host in FP64 and kept on the
// device in both precisions; the kernel forms values[v][q][i] =
// sum_l phi[q][l] coeffs[v][l][i], one lane per cell, reading each cell's
// coefficients once and writing each value once (HBM-bound: no data reuse
// across cells, so no MFMA).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "cweno.h"
#include "host.hpp"
#include "dispatch.hpp"
#include "mesh.hpp"
#include "reconstruct_kernel.hpp"

struct cweno_points {
  int d = 2, M = 1, n = 0, device = -1;
  std::vector<double> phi;         // host copy [n][nb]
  cweno_abi::DevBuf phi64, phi32;
  ~cweno_points() {
    if (phi64.p) (void)hipFree(phi64.p);
    if (phi32.p) (void)hipFree(phi32.p);
  }
};

namespace cweno {

template <typename T>
struct EParams {
  const T* coeffs;   // [nv][NB][nc]
  T* values;         // [nv][np][nc]
  const T* phi;      // [np][NB]
  int64_t nc;
  int nv, np;
};

template <int D, int M, typename T>
__global__ __launch_bounds__(kThreads) void evaluate_kernel(EParams<T> p, const T* __restrict__ coeffs,
                                                            T* __restrict__ values, const T* __restrict__ phi) {
  constexpr int NB = nbasis_c(M, D);
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (i >= p.nc) return;
  const int64_t nc = p.nc;
  for (int v = 0; v < p.nv; ++v) {
    const T* c = coeffs + (int64_t)v * NB * nc + i;
    T cv[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) cv[l] = __builtin_nontemporal_load(c + (int64_t)l * nc);
    T* o = values + (int64_t)v * p.np * nc + i;
    for (int q = 0; q < p.np; ++q) {
      const T* f = phi + q * NB;
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NB; ++l) s = fma(f[l], cv[l], s);
      __builtin_nontemporal_store(s, o + (int64_t)q * nc);
    }
  }
}

template <typename T>
hipError_t launch_evaluate(int d, int M, const EParams<T>& p, hipStream_t s) {
  const unsigned blocks = (unsigned)((p.nc + kThreads - 1) / kThreads);
#define CWENO_EVAL_CASE(DD, MM)                                                                       \
  case DD * 10 + MM:                                                                                  \
    hipLaunchKernelGGL((evaluate_kernel<DD, MM, T>), dim3(blocks), dim3(kThreads), 0, s, p, p.coeffs, \
                       p.values, p.phi);                                                              \
    return hipGetLastError();
  switch (d * 10 + M) {
    CWENO_EVAL_CASE(2, 1) CWENO_EVAL_CASE(2, 2) CWENO_EVAL_CASE(2, 3) CWENO_EVAL_CASE(2, 4)
    CWENO_EVAL_CASE(3, 1) CWENO_EVAL_CASE(3, 2) CWENO_EVAL_CASE(3, 3) CWENO_EVAL_CASE(3, 4)
  }
#undef CWENO_EVAL_CASE
  return hipErrorInvalidValue;
}

}  // namespace cweno

using cweno_abi::fail;
using cweno_abi::overlap;

namespace {

cweno_status to_device(cweno_abi::DevBuf& b, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(CWENO_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  b.bytes = bytes;
  e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipMemcpy failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

}  // namespace

extern "C" {

cweno_status cweno_points_create(int dim, int degree, int n_points, const double* ref_points, cweno_points** out) {
  if (!out) return fail(CWENO_E_ARG, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(CWENO_E_ARG, "dim must be 2 or 3");
  if (degree < 1 || degree > 4) return fail(CWENO_E_ARG, "degree must be in 1..4");
  if (n_points < 1 || n_points > 4096 || !ref_points) return fail(CWENO_E_ARG, "need 1..4096 points");
  for (int k = 0; k < n_points * dim; ++k)
    if (!std::isfinite(ref_points[k])) return fail(CWENO_E_ARG, "reference points must be finite");
  std::unique_ptr<cweno_points> P(new (std::nothrow) cweno_points());
  if (!P) return fail(CWENO_E_NOMEM, "host allocation failed");
  P->d = dim;
  P->M = degree;
  P->n = n_points;
  const int nb = cweno::n_basis(degree, dim);
  P->phi.resize((size_t)n_points * nb);
  try {
    for (int q = 0; q < n_points; ++q) cweno::basis_eval(dim, degree, ref_points + (size_t)q * dim, &P->phi[(size_t)q * nb]);
  } catch (const cweno::Error& e) {
    return fail(e.code, e.what());
  }
  if (hipGetDevice(&P->device) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
  std::vector<float> f32(P->phi.begin(), P->phi.end());
  if (cweno_status st = to_device(P->phi64, P->phi.data(), P->phi.size() * 8)) return st;
  if (cweno_status st = to_device(P->phi32, f32.data(), f32.size() * 4)) return st;
  *out = P.release();
  return CWENO_OK;
}

cweno_status cweno_points_destroy(cweno_points* p) {
  delete p;
  return CWENO_OK;
}

cweno_status cweno_points_basis(const cweno_points* p, double* phi) {
  if (!p || !phi) return fail(CWENO_E_ARG, "points and phi are required");
  std::copy(p->phi.begin(), p->phi.end(), phi);
  return CWENO_OK;
}

cweno_status cweno_reconstruct_points(const cweno_mesh* m, const cweno_points* pts, int n_vars, cweno_dtype dtype,
                                      const void* q, void* values, void* hip_stream) {
  if (!m || !pts) return fail(CWENO_E_ARG, "mesh and points are required");
  if (pts->d != m->d || pts->M != m->M) return fail(CWENO_E_ARG, "point set built for another dimension or degree");
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!q || !values) return fail(CWENO_E_ARG, "q and values must be device pointers");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  if (m->n_s > 0) return fail(CWENO_E_ARG, "a WENO mesh has no fused point values (reconstruct, then evaluate)");
  const bool f32 = dtype == CWENO_F32;
  if ((f32 && !m->pinv32.p) || (!f32 && !m->pinv64.p))
    return fail(CWENO_E_ARG, "the mesh holds no operators of this precision");
  if (m->maxH <= 0) return fail(CWENO_E_ARG, "fused point values need the LDS-halo kernel, which this mesh cannot use");
  const uint64_t es = f32 ? 4 : 8, cells = (uint64_t)m->nc * (uint64_t)n_vars;
  if ((uint64_t)pts->n * (uint64_t)m->nc * es >= (uint64_t(1) << 32) ||
      (uint64_t)m->nc * (uint64_t)m->nb * es >= (uint64_t(1) << 32))
    return fail(CWENO_E_ARG, "too many cells or points for 32-bit offsets within one variable's values");
  if (overlap(q, cells * es, values, cells * (uint64_t)pts->n * es))
    return fail(CWENO_E_ARG, "q and values must not overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  for (int v0 = 0; v0 < n_vars;) {
    int vb = cweno::pick_vb_one_pass(m->d, m->M, n_vars - v0, f32);
    // the block halo of vb variables and a column of nb-1 coefficients per thread must fit in LDS
    const int64_t col = (int64_t)(m->nb - 1) * cweno::kHaloBlock * (int64_t)es;
    while (vb > 1 && (int64_t)m->maxH * vb * (int64_t)es + col > cweno::kMaxLds)
      vb = cweno::pick_vb_one_pass(m->d, m->M, vb - 1, f32);
    if ((int64_t)m->maxH * vb * (int64_t)es + col > cweno::kMaxLds)
      return fail(CWENO_E_ARG, "the block halos of this mesh leave no room for the fused point values");
    hipError_t e;
    if (f32) {
      cweno::KParams<float> p = cweno_abi::make_params<float>(m, q, nullptr, nullptr, nullptr, v0);
      p.phi = (const float*)pts->phi32.p;
      p.pv = (float*)values;
      p.npts = pts->n;
      e = cweno::launch_points<float>(m->d, m->M, p, vb, s);
    } else {
      cweno::KParams<double> p = cweno_abi::make_params<double>(m, q, nullptr, nullptr, nullptr, v0);
      p.phi = (const double*)pts->phi64.p;
      p.pv = (double*)values;
      p.npts = pts->n;
      e = cweno::launch_points<double>(m->d, m->M, p, vb, s);
    }
    if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    v0 += vb;
  }
  return CWENO_OK;
}

cweno_status cweno_evaluate(const cweno_mesh* m, const cweno_points* pts, int n_vars, cweno_dtype dtype,
                            const void* coeffs, void* values, void* hip_stream) {
  if (!m || !pts) return fail(CWENO_E_ARG, "mesh and points are required");
  if (pts->d != m->d || pts->M != m->M) return fail(CWENO_E_ARG, "point set built for another dimension or degree");
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!coeffs || !values) return fail(CWENO_E_ARG, "coeffs and values must be device pointers");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  const bool f32 = dtype == CWENO_F32;
  const uint64_t es = f32 ? 4 : 8, cells = (uint64_t)m->nc * (uint64_t)n_vars;
  if (overlap(coeffs, cells * (uint64_t)m->nb * es, values, cells * (uint64_t)pts->n * es))
    return fail(CWENO_E_ARG, "coeffs and values must not overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e;
  if (f32) {
    cweno::EParams<float> p{(const float*)coeffs, (float*)values, (const float*)pts->phi32.p, m->nc, n_vars, pts->n};
    e = cweno::launch_evaluate<float>(m->d, m->M, p, s);
  } else {
    cweno::EParams<double> p{(const double*)coeffs, (double*)values, (const double*)pts->phi64.p, m->nc, n_vars,
                             pts->n};
    e = cweno::launch_evaluate<double>(m->d, m->M, p, s);
  }
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

}  // extern "C"
