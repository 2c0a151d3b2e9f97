// Basis matrix of the expansion (Sec. II-A): Psi[v][col] = h^3 * real columns
// of conj(psi_klm) at the orbit representatives of the ball voxels (divided
// by the size of the voxel's stabiliser under the three coordinate
// reflections: 1 unless the voxel lies on a mirror plane of an odd grid),
// built once per plan in FP64 and rounded to FP32.
//
// Real columns of radial entry (l, k), j = 0..2l: j = 0 -> conj(psi_kl0)
// (real); j = 2m - 1 -> Re conj(psi_klm); j = 2m -> Im conj(psi_klm),
// m = 1..l.  For real f the complex coefficients follow from these
// (a_{k,l,-m} = (-1)^m conj(a_klm)).  The columns are stored grouped by
// parity class (column_parity_class), each class padded to whole tiles.
//
// Y_l^m = Pbar_l^m(cos theta) e^{i m phi} with the normalised associated
// Legendre functions (Condon-Shortley phase), computed by the standard
// recurrences in l:
//   Pbar_0^0 = 1/sqrt(4 pi),  Pbar_m^m = -sqrt((2m+1)/(2m)) sin(theta) Pbar_{m-1}^{m-1},
//   Pbar_{m+1}^m = sqrt(2m+3) cos(theta) Pbar_m^m,
//   Pbar_l^m = a_lm (cos(theta) Pbar_{l-1}^m - b_lm Pbar_{l-2}^m),
//   a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
#include "bh_internal.h"
#include "bh_special.h"

#include <cmath>

namespace bh {
namespace {

__device__ inline void voxel_coords(int32_t lin, int N, double& x, double& y, double& z) {
  const int k = lin % N;
  const int j = (lin / N) % N;
  const int i = lin / (N * N);
  const double h = 2.0 / N;
  x = (i - 0.5 * (N - 1)) * h;
  y = (j - 0.5 * (N - 1)) * h;
  z = (k - 0.5 * (N - 1)) * h;
}

// Real spherical-harmonic table of a chunk of voxels: thread per (voxel, m).
// Yr[v][l*l + j]: j = 0 -> Y_l^0; j = 2m-1 -> Re Y_l^m; j = 2m -> Im conj Y_l^m.
__global__ void k_ylm(const int32_t* __restrict__ vidx, int64_t v0, int64_t nv, int N, int L,
                      double* __restrict__ Yr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vl = t / (L + 1);
  const int m = (int)(t % (L + 1));
  if (vl >= nv) return;
  double x, y, z;
  voxel_coords(vidx[v0 + vl], N, x, y, z);
  const double r = sqrt(x * x + y * y + z * z);
  const double ct = (r > 0) ? z / r : 1.0;
  const double st = (r > 0) ? sqrt(x * x + y * y) / r : 0.0;
  const double phi = atan2(y, x);
  double cm, sm;
  sincos(m * phi, &sm, &cm);
  const int64_t stride = (int64_t)(L + 1) * (L + 1);
  double* row = Yr + vl * stride;
  double pmm = 0.28209479177387814347;   // 1/sqrt(4 pi)
  for (int i = 1; i <= m; ++i) pmm *= -sqrt((2.0 * i + 1.0) / (2.0 * i)) * st;
  auto put = [&](int l, double P) {
    if (m == 0) {
      row[l * l] = P;
    } else {
      row[l * l + 2 * m - 1] = P * cm;
      row[l * l + 2 * m] = -P * sm;
    }
  };
  put(m, pmm);
  if (m + 1 > L) return;
  double p1 = sqrt(2.0 * m + 3.0) * ct * pmm;   // l = m + 1
  put(m + 1, p1);
  double p0 = pmm;
  for (int l = m + 2; l <= L; ++l) {
    const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
    const double b = sqrt((((double)l - 1) * (l - 1) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
    const double p2 = a * (ct * p1 - b * p0);
    put(l, p2);
    p0 = p1;
    p1 = p2;
  }
}

// Radial table Rt[v][e] = c_e j_{l_e}(lambda_e r_v): thread per (voxel, entry).
__global__ void k_radial(const int32_t* __restrict__ vidx, int64_t v0, int64_t nv, int N,
                         const int32_t* __restrict__ ent_l, const double* __restrict__ ent_lam,
                         const double* __restrict__ ent_c, int n_ent, double* __restrict__ Rt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vl = t / n_ent;
  const int e = (int)(t % n_ent);
  if (vl >= nv) return;
  double x, y, z;
  voxel_coords(vidx[v0 + vl], N, x, y, z);
  const double r = sqrt(x * x + y * y + z * z);
  Rt[vl * n_ent + e] = ent_c[e] * bh_sph_jn(ent_l[e], ent_lam[e] * r);
}

// Psi[v0 + vl][col] for a chunk of representatives; padding rows and
// columns (col_ent < 0) are zero.
__global__ void k_psi_fill(int64_t v0, int64_t nv, int64_t VR, int64_t C_pad, int N, int L,
                           double h3, const int32_t* __restrict__ vrep,
                           const int32_t* __restrict__ col_ent, const int32_t* __restrict__ col_y,
                           int n_ent, const double* __restrict__ Rt, const double* __restrict__ Yr,
                           float* __restrict__ psi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vl = t / C_pad;
  const int64_t col = t % C_pad;
  if (vl >= nv) return;
  const int64_t v = v0 + vl;
  float val = 0.0f;
  const int32_t e = col_ent[col];
  if (v < VR && e >= 0) {
    const int32_t lin = vrep[v];
    // a coordinate on a mirror plane (odd grid, index (N-1)/2) halves the orbit
    double w = h3;
    if (2 * (lin / (N * N)) == N - 1) w *= 0.5;
    if (2 * ((lin / N) % N) == N - 1) w *= 0.5;
    if (2 * (lin % N) == N - 1) w *= 0.5;
    const int64_t ys = (int64_t)(L + 1) * (L + 1);
    val = (float)(w * Rt[vl * n_ent + e] * Yr[vl * ys + col_y[col]]);
  }
  psi[v * C_pad + col] = val;
}

template <typename T>
int upload(const std::vector<T>& h, T** d) {
  *d = nullptr;
  if (h.empty()) return BH_OK;
  BH_HIP(hipMalloc((void**)d, h.size() * sizeof(T)));
  BH_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return BH_OK;
}

}  // namespace

int build_basis(bh_plan* p) {
  const IndexSet& idx = *p->idx;
  const int L = p->L_max;
  const int n_ent = (int)idx.rad.size();
  std::vector<int32_t> vox = orbit_representatives(p->N);
  p->V = (int64_t)ball_voxels(p->N).size();
  p->VR = (int64_t)vox.size();
  p->VR_pad = ((p->VR + kGemmKAlign - 1) / kGemmKAlign) * kGemmKAlign;
  p->C = idx.C;

  // stored position of every real column: class after class, each class
  // padded to whole tiles
  std::vector<int32_t> ccls(p->C);
  int64_t ccount[kParityClasses] = {};
  for (const Radial& r : idx.rad)
    for (int j = 0; j <= 2 * r.l; ++j) ++ccount[ccls[r.offset + j] = column_parity_class(r.l, j)];
  int64_t cnext[kParityClasses];
  p->ctiles.first[0] = 0;
  for (int c = 0; c < kParityClasses; ++c) {
    cnext[c] = (int64_t)p->ctiles.first[c] * kGemmBN;
    p->ctiles.first[c + 1] = p->ctiles.first[c] + (int32_t)((ccount[c] + kGemmBN - 1) / kGemmBN);
  }
  p->C_pad = (int64_t)p->ctiles.first[kParityClasses] * kGemmBN;
  std::vector<int32_t> pos(p->C);
  for (int64_t col = 0; col < p->C; ++col) pos[col] = (int32_t)cnext[ccls[col]]++;

  // per stored column tables and the complex-coefficient source map
  std::vector<int32_t> col_ent(p->C_pad, -1), col_y(p->C_pad, 0), csrc(2 * p->C);
  std::vector<float> csgn(2 * p->C);
  std::vector<int32_t> e_l(n_ent);
  std::vector<double> e_lam(n_ent), e_c(n_ent);
  for (int e = 0; e < n_ent; ++e) {
    const Radial& r = idx.rad[e];
    e_l[e] = r.l;
    e_lam[e] = r.lam;
    e_c[e] = r.c;
    for (int j = 0; j <= 2 * r.l; ++j) {
      col_ent[pos[r.offset + j]] = e;
      col_y[pos[r.offset + j]] = r.l * r.l + j;
    }
    for (int m = -r.l; m <= r.l; ++m) {
      const int q = r.offset + r.l + m;
      const int am = m < 0 ? -m : m;
      const float sg = (m < 0 && (am % 2)) ? -1.0f : 1.0f;   // (-1)^m for m < 0
      if (am == 0) {
        csrc[2 * q] = pos[r.offset]; csgn[2 * q] = 1.0f;
        csrc[2 * q + 1] = -1;        csgn[2 * q + 1] = 0.0f;
      } else {
        csrc[2 * q] = pos[r.offset + 2 * am - 1];
        csgn[2 * q] = sg;
        csrc[2 * q + 1] = pos[r.offset + 2 * am];
        csgn[2 * q + 1] = (m < 0) ? -sg : 1.0f;                // conj for m < 0
      }
    }
  }
  int rc;
  if ((rc = upload(vox, &p->vrep)) != BH_OK) return rc;
  if ((rc = upload(csrc, &p->csrc)) != BH_OK) return rc;
  if ((rc = upload(csgn, &p->csgn)) != BH_OK) return rc;
  int32_t *d_col_ent = nullptr, *d_col_y = nullptr, *d_el = nullptr;
  double *d_elam = nullptr, *d_ec = nullptr, *d_Rt = nullptr, *d_Yr = nullptr;
  struct Cleanup {
    std::vector<void*> ptrs;
    ~Cleanup() { for (void* q : ptrs) if (q) (void)hipFree(q); }
  } cleanup;
  if ((rc = upload(col_ent, &d_col_ent)) != BH_OK) return rc;
  cleanup.ptrs.push_back(d_col_ent);
  if ((rc = upload(col_y, &d_col_y)) != BH_OK) return rc;
  cleanup.ptrs.push_back(d_col_y);
  if ((rc = upload(e_l, &d_el)) != BH_OK) return rc;
  cleanup.ptrs.push_back(d_el);
  if ((rc = upload(e_lam, &d_elam)) != BH_OK) return rc;
  cleanup.ptrs.push_back(d_elam);
  if ((rc = upload(e_c, &d_ec)) != BH_OK) return rc;
  cleanup.ptrs.push_back(d_ec);

  const size_t psi_bytes = (size_t)p->VR_pad * p->C_pad * sizeof(float);
  if (hipMalloc((void**)&p->psi, psi_bytes) != hipSuccess) {
    p->psi = nullptr;
    return set_error(BH_ENOMEM, "basis matrix allocation failed");
  }
  // voxel chunks bound the FP64 temporaries to ~1 GiB
  const int64_t ys = (int64_t)(L + 1) * (L + 1);
  int64_t chunk = (int64_t)1 << 30;
  chunk /= (int64_t)sizeof(double) * (ys + n_ent);
  chunk = chunk < 1024 ? 1024 : chunk;
  chunk = chunk > p->VR_pad ? p->VR_pad : chunk;
  BH_HIP(hipMalloc((void**)&d_Yr, (size_t)chunk * ys * sizeof(double)));
  cleanup.ptrs.push_back(d_Yr);
  BH_HIP(hipMalloc((void**)&d_Rt, (size_t)chunk * (n_ent > 0 ? n_ent : 1) * sizeof(double)));
  cleanup.ptrs.push_back(d_Rt);
  const double h = 2.0 / p->N;
  const double h3 = h * h * h;
  for (int64_t v0 = 0; v0 < p->VR_pad; v0 += chunk) {
    const int64_t nv = (v0 + chunk <= p->VR_pad) ? chunk : p->VR_pad - v0;
    const int64_t nreal = (v0 >= p->VR) ? 0 : ((v0 + nv <= p->VR) ? nv : p->VR - v0);
    if (nreal > 0) {
      const int64_t t1 = nreal * (L + 1);
      hipLaunchKernelGGL(k_ylm, dim3((unsigned)((t1 + 255) / 256)), dim3(256), 0, 0, p->vrep, v0,
                         nreal, p->N, L, d_Yr);
      BH_HIP(hipGetLastError());
      if (n_ent > 0) {
        const int64_t t2 = nreal * n_ent;
        hipLaunchKernelGGL(k_radial, dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, 0, p->vrep,
                           v0, nreal, p->N, d_el, d_elam, d_ec, n_ent, d_Rt);
        BH_HIP(hipGetLastError());
      }
    }
    const int64_t t3 = nv * p->C_pad;
    hipLaunchKernelGGL(k_psi_fill, dim3((unsigned)((t3 + 255) / 256)), dim3(256), 0, 0, v0, nv,
                       p->VR, p->C_pad, p->N, L, h3, p->vrep, d_col_ent, d_col_y,
                       n_ent > 0 ? n_ent : 1, d_Rt, d_Yr, p->psi);
    BH_HIP(hipGetLastError());
  }
  BH_HIP(hipDeviceSynchronize());
  return BH_OK;
}

}  // namespace bh
