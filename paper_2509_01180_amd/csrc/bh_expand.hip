// Expansion (Sec. II-A): a[b][c] = sum_v F[b][v] Psi[v][c], the voxel
// quadrature of <f, psi_klm> as dense real GEMMs on MFMA, then the complex
// coefficients of every m are rebuilt from the real columns.
//
// The sum runs over orbit representatives of the three coordinate
// reflections, one GEMM slice per parity class of the columns (the fold is
// described with ClassTiles).
//
//   k_gather  : volumes [B][N^3] -> Ft[8][VR_pad][M_pad]: the 8 signed
//               mirror sums g_P of each representative, transposed and zero
//               padded, so both GEMM operands are K-major.
//   k_gemm_f32: split-K GEMM on v_mfma_f32_32x32x2f32, 128x128 tiles,
//               K step 32, LDS double buffer; partial sums per split; a
//               column tile reads the Ft slice of its class.
//   k_reduce  : sums the splits in a fixed order and writes the complex
//               layout (re, im) for m = -l..l.
#include "bh_internal.h"

#include <algorithm>
#include <mutex>

// Device scratch of the allocation-free expansion (bh_expand_noalloc): the
// folded volumes and split-K partial sums of one pass.  Every GPU the
// library runs on holds one copy for the life of the process.  Host code
// never uses this name as an address: each device's copy is resolved once
// with hipGetSymbolAddress (noalloc_scratch_init) and only that pointer is
// handed to kernels.
static __device__ __align__(256) float scratch[BH_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace bh {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;

// Ft[P][v][b] = g_P of particle b at representative v (0 outside v < VR,
// b < B).  32x32 LDS transpose per class.  Particle b's volume is
// vols[rows[b]] with a row table (a row outside [0, n_rows) reads as NaN
// and raises the error word `bad`), else vols[b].
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ vols, int64_t vol_stride,
                                                int64_t B, const int64_t* __restrict__ rows,
                                                int64_t n_rows, int* bad,
                                                const int32_t* __restrict__ vrep,
                                                int64_t VR, int64_t VR_pad, int64_t M_pad, int N,
                                                float* __restrict__ Ft) {
  __shared__ float tile[kParityClasses][32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t v0 = (int64_t)blockIdx.x * 32, b0 = (int64_t)blockIdx.y * 32;
  const int64_t v = v0 + tx;
  int32_t off[8];
  mirror_offsets((v < VR) ? vrep[v] : 0, N, off);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t b = b0 + ty + 8 * i;
    float f[8];
    const int64_t r = volume_row(rows, n_rows, B, b, v == 0 ? bad : nullptr);
    const bool in = v < VR && r >= 0;
    const float* vb = vols + (in ? r * vol_stride : 0);
    const float outside = r == -2 ? __builtin_nanf("") : 0.0f;
#pragma unroll
    for (int s = 0; s < 8; ++s) f[s] = in ? vb[off[s]] : outside;
    parity_fold(f);
#pragma unroll
    for (int c = 0; c < kParityClasses; ++c) tile[c][ty + 8 * i][tx] = f[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kParityClasses; ++c) {
    float* out = Ft + (int64_t)c * VR_pad * M_pad;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t vv = v0 + ty + 8 * i;
      out[vv * M_pad + b0 + tx] = tile[c][tx][ty + 8 * i];
    }
  }
}

// As k_gather for rows r = b * S + s of integer-shifted volumes: the images
// are taken of f_b moved by shift s, i.e. vols[b][i + dx][j + dy][k + dz]
// at image (i, j, k) (0 where that leaves the box).
__global__ __launch_bounds__(256) void k_gather_shift(const float* __restrict__ vols, int N,
                                                      int64_t rows, int S, ShiftTable shifts,
                                                      const int32_t* __restrict__ vrep, int64_t VR,
                                                      int64_t VR_pad, int64_t M_pad,
                                                      float* __restrict__ Ft) {
  __shared__ float tile[kParityClasses][32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t v0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int64_t v = v0 + tx;
  const int32_t lin = (v < VR) ? vrep[v] : 0;
  const int vi = lin / (N * N), vj = (lin / N) % N, vk = lin % N;
  const int64_t vol_stride = (int64_t)N * N * N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty + 8 * i;
    float f[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) f[s] = 0.0f;
    if (v < VR && r < rows) {
      const int64_t b = r / S;
      const int sh = (int)(r % S);
      const float* vb = vols + b * vol_stride;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int si = ((s & 1) ? N - 1 - vi : vi) + shifts.d[sh][0];
        const int sj = ((s & 2) ? N - 1 - vj : vj) + shifts.d[sh][1];
        const int sk = ((s & 4) ? N - 1 - vk : vk) + shifts.d[sh][2];
        if (si >= 0 && si < N && sj >= 0 && sj < N && sk >= 0 && sk < N)
          f[s] = vb[((int64_t)si * N + sj) * N + sk];
      }
    }
    parity_fold(f);
#pragma unroll
    for (int c = 0; c < kParityClasses; ++c) tile[c][ty + 8 * i][tx] = f[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kParityClasses; ++c) {
    float* out = Ft + (int64_t)c * VR_pad * M_pad;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t vv = v0 + ty + 8 * i;
      out[vv * M_pad + r0 + tx] = tile[c][tx][ty + 8 * i];
    }
  }
}

// part[s][m][n] = sum_{k in split s} Ft[k][m] Psi[k][n].
// 4 waves in a 2x2 arrangement, each 64x64 = 2x2 MFMA 32x32 tiles.
// MFMA 32x32x2 f32 operand layout: lane L supplies A[L%32][L/32] and
// B[L/32][L%32]; accumulator r of lane L is D[8(r/4) + 4(L/32) + r%4][L%32].
__global__ __launch_bounds__(256, 2) void k_gemm_f32(const float* __restrict__ Ft,
                                                     const float* __restrict__ Psi,
                                                     float* __restrict__ part, int64_t M_pad,
                                                     int64_t C_pad, int64_t VR_pad, ClassTiles ct,
                                                     int64_t nk_total, int nsplit) {
  __shared__ float As[2][BK][BM];
  __shared__ float Bs[2][BK][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t tm, tn, ts;
  gemm_tile(blockIdx.x, M_pad / BM, C_pad / BN, nsplit, tm, tn, ts);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  int64_t k0, nk64;
  split_range(ts, nsplit, nk_total, k0, nk64);
  const int nk = (int)nk64;
  const int64_t k_begin = k0 * BK;
  const int lr = tid >> 5, lc = (tid & 31) * 4;
  const float* pa = Ft + class_of_tile(ct, tn) * VR_pad * M_pad + (k_begin + lr) * M_pad + m0 + lc;
  const float* pb = Psi + (k_begin + lr) * C_pad + n0 + lc;
  const int64_t sa = 8 * M_pad, sb = 8 * C_pad;          // 8 rows apart
  const int64_t stepa = BK * M_pad, stepb = BK * C_pad;  // one K step
  float4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define BH_GLOAD(kt)                                                        \
  do {                                                                      \
    const float* qa = pa + (int64_t)(kt) * stepa;                           \
    const float* qb = pb + (int64_t)(kt) * stepb;                           \
    ra0 = *reinterpret_cast<const float4*>(qa);                             \
    ra1 = *reinterpret_cast<const float4*>(qa + sa);                        \
    ra2 = *reinterpret_cast<const float4*>(qa + 2 * sa);                    \
    ra3 = *reinterpret_cast<const float4*>(qa + 3 * sa);                    \
    rb0 = *reinterpret_cast<const float4*>(qb);                             \
    rb1 = *reinterpret_cast<const float4*>(qb + sb);                        \
    rb2 = *reinterpret_cast<const float4*>(qb + 2 * sb);                    \
    rb3 = *reinterpret_cast<const float4*>(qb + 3 * sb);                    \
  } while (0)
#define BH_SSTORE(buf)                                                      \
  do {                                                                      \
    *reinterpret_cast<float4*>(&As[buf][lr][lc]) = ra0;                     \
    *reinterpret_cast<float4*>(&As[buf][lr + 8][lc]) = ra1;                 \
    *reinterpret_cast<float4*>(&As[buf][lr + 16][lc]) = ra2;                \
    *reinterpret_cast<float4*>(&As[buf][lr + 24][lc]) = ra3;                \
    *reinterpret_cast<float4*>(&Bs[buf][lr][lc]) = rb0;                     \
    *reinterpret_cast<float4*>(&Bs[buf][lr + 8][lc]) = rb1;                 \
    *reinterpret_cast<float4*>(&Bs[buf][lr + 16][lc]) = rb2;                \
    *reinterpret_cast<float4*>(&Bs[buf][lr + 24][lc]) = rb3;                \
  } while (0)
  floatx16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int hl = lane >> 5, ll = lane & 31;
  BH_GLOAD(0);
  BH_SSTORE(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) BH_GLOAD(kt + 1);
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int k = 2 * kk + hl;
      const float a0 = As[cur][k][wm + ll], a1 = As[cur][k][wm + 32 + ll];
      const float b0 = Bs[cur][k][wn + ll], b1 = Bs[cur][k][wn + 32 + ll];
      acc00 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc11, 0, 0, 0);
    }
    if (kt + 1 < nk) BH_SSTORE(cur ^ 1);
    __syncthreads();
  }
#undef BH_GLOAD
#undef BH_SSTORE
  float* out = part + ts * M_pad * C_pad;
  const int64_t row0 = m0 + wm + 4 * hl, col0 = n0 + wn + ll;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = row0 + 8 * (r >> 2) + (r & 3);
    out[row * C_pad + col0] = acc00[r];
    out[row * C_pad + col0 + 32] = acc01[r];
    out[(row + 32) * C_pad + col0] = acc10[r];
    out[(row + 32) * C_pad + col0 + 32] = acc11[r];
  }
}

// coeffs[b][q] = (sum_s part[s][b][src_re] * sgn_re, sum_s part[s][b][src_im] * sgn_im)
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ part, int nsplit,
                                                int64_t M_pad, int64_t C_pad, int64_t B, int64_t C,
                                                const int32_t* __restrict__ csrc,
                                                const float* __restrict__ csgn,
                                                float* __restrict__ coeffs, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * C) return;
  const int64_t b = t / C, q = t % C;
  const int32_t sr = csrc[2 * q], si = csrc[2 * q + 1];
  // every split's loads first (in flight together), then the sums in split order
  float vr[kMaxSplit], vi[kMaxSplit];
#pragma unroll
  for (int s = 0; s < kMaxSplit; ++s) {
    if (s < nsplit) {
      const float* ps = part + (int64_t)s * M_pad * C_pad + b * C_pad;
      vr[s] = ps[sr];
      vi[s] = si >= 0 ? ps[si] : 0.0f;
    }
  }
  float re = 0.0f, im = 0.0f;
#pragma unroll
  for (int s = 0; s < kMaxSplit; ++s) {
    if (s < nsplit) {
      re += vr[s];
      im += vi[s];
    }
  }
  const int64_t o = b * ldc + q;
  coeffs[2 * o] = re * csgn[2 * q];
  coeffs[2 * o + 1] = (si >= 0) ? im * csgn[2 * q + 1] : 0.0f;
}

}  // namespace

int launch_expand(bh_plan* p, const float* vols, int64_t B, float* coeffs, hipStream_t s,
                  bool batch_invariant, const ShiftTable* shifts, int S, int64_t ldc,
                  const int64_t* rows, int64_t n_rows) {
  if (ldc <= 0) ldc = p->C;
  if (shifts) B *= S;   // one GEMM row per (particle, shift)
  if (B == 0) return BH_OK;
  const int64_t M_pad = ((B + BM - 1) / BM) * BM;
  const int64_t mt = M_pad / BM, nt = p->C_pad / BN;
  const int64_t nk_total = p->VR_pad / BK;          // multiple of 16
  const int nsplit = expand_split_f32(p, B, batch_invariant);
  int rc;
  if ((rc = grow(p->gathered, (size_t)kParityClasses * p->VR_pad * M_pad * sizeof(float))) != BH_OK)
    return rc;
  if ((rc = grow(p->partial, (size_t)nsplit * M_pad * p->C_pad * sizeof(float))) != BH_OK) return rc;
  float* Ft = (float*)p->gathered.ptr;
  float* part = (float*)p->partial.ptr;
  const int64_t vol_stride = (int64_t)p->N * p->N * p->N;
  if (shifts) {
    ProfScope ps(p, "gather_shift", s, B);
    hipLaunchKernelGGL(k_gather_shift, dim3((unsigned)(p->VR_pad / 32), (unsigned)(M_pad / 32)),
                       dim3(256), 0, s, vols, p->N, B, S, *shifts, p->vrep, p->VR, p->VR_pad,
                       M_pad, Ft);
  } else {
    ProfScope ps(p, "gather", s, B);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)(p->VR_pad / 32), (unsigned)(M_pad / 32)),
                       dim3(256), 0, s, vols, vol_stride, B, rows, n_rows, p->err_dev, p->vrep,
                       p->VR, p->VR_pad, M_pad, p->N, Ft);
  }
  BH_HIP(hipGetLastError());
  {
  ProfScope ps(p, "gemm", s, B);
  hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)(mt * nt * nsplit)), dim3(256), 0, s, Ft, p->psi,
                     part, M_pad, p->C_pad, p->VR_pad, p->ctiles, nk_total, nsplit);
  }
  BH_HIP(hipGetLastError());
  const int64_t tot = B * p->C;
  {
  ProfScope ps(p, "reduce", s, B);
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part, nsplit,
                     M_pad, p->C_pad, B, p->C, p->csrc, p->csgn, coeffs, ldc);
  }
  BH_HIP(hipGetLastError());
  return BH_OK;
}

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices)
    return set_error(BH_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return BH_OK;
  int cur = -1;
  BH_HIP(hipGetDevice(&cur));
  if (cur != device) return set_error(BH_EDEVICE, "scratch lookup needs its device current");
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_error(BH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
  }
  g_scratch_ptr[device] = ptr;
  return BH_OK;
}

int noalloc_expand_pass(const bh_plan* p, int64_t* tiles_per_pass) {
  const int64_t nt = p->C_pad / BN, nk_total = p->VR_pad / BK;
  const int nsplit = expand_split(1, nt, nk_total, true);
  const size_t ft_tile = (size_t)kParityClasses * p->VR_pad * BM * sizeof(float);
  const size_t part_tile = (size_t)nsplit * BM * p->C_pad * sizeof(float);
  *tiles_per_pass = (int64_t)(BH_NOALLOC_SCRATCH_BYTES / (ft_tile + part_tile));
  return nsplit;
}

// bh_expand_noalloc: the batch-invariant FP32 expansion (the same kernels,
// split and summation order as launch_expand with batch_invariant) in passes
// of whole 128-particle tiles whose folded volumes and partial sums fit the
// static scratch.  Allocates nothing; the scratch needs no clearing (the
// gather writes every folded value, padding included, and the GEMM every
// partial sum before they are read).
int launch_expand_noalloc(bh_plan* p, const float* vols, int64_t B, float* coeffs,
                          hipStream_t s) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (p->device >= 0 && p->device < kMaxScratchDevices) base = g_scratch_ptr[p->device];
  }
  if (!base) return set_error(BH_EDEVICE, "scratch of this device not resolved");
  int64_t tiles_per_pass = 0;
  const int nsplit = noalloc_expand_pass(p, &tiles_per_pass);
  if (tiles_per_pass < 1)
    return set_error(BH_EUNSUPPORTED, "one 128-particle tile of this plan needs more than the " +
                                          std::to_string(BH_NOALLOC_SCRATCH_BYTES >> 20) +
                                          " MiB scratch");
  const int64_t nt = p->C_pad / BN, nk_total = p->VR_pad / BK;
  const int64_t vol_stride = (int64_t)p->N * p->N * p->N;
  for (int64_t b0 = 0; b0 < B; b0 += tiles_per_pass * BM) {
    const int64_t nb = std::min(B - b0, tiles_per_pass * BM);
    const int64_t M_pad = ((nb + BM - 1) / BM) * BM, mt = M_pad / BM;
    float* Ft = (float*)base;
    float* part = Ft + (size_t)kParityClasses * p->VR_pad * M_pad;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)(p->VR_pad / 32), (unsigned)(M_pad / 32)),
                       dim3(256), 0, s, vols + b0 * vol_stride, vol_stride, nb, nullptr, 0,
                       nullptr, p->vrep, p->VR, p->VR_pad, M_pad, p->N, Ft);
    BH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)(mt * nt * nsplit)), dim3(256), 0, s, Ft,
                       p->psi, part, M_pad, p->C_pad, p->VR_pad, p->ctiles, nk_total, nsplit);
    BH_HIP(hipGetLastError());
    const int64_t tot = nb * p->C;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part,
                       nsplit, M_pad, p->C_pad, nb, p->C, p->csrc, p->csgn,
                       coeffs + 2 * b0 * p->C, p->C);
    BH_HIP(hipGetLastError());
  }
  return BH_OK;
}

// q = 4: a tile's 64 KB of partial sums, written and read back, against the
// chip-wide time of a K-step of 32 KB of operands (about 3.8 us per workgroup).
int expand_split_f32(const bh_plan* p, int64_t B, bool batch_invariant) {
  const int64_t mt = (B + BM - 1) / BM, nt = p->C_pad / BN, nk_total = p->VR_pad / BK;
  return expand_split(mt, nt, nk_total, batch_invariant, &p->tuned_split[0],
                      batch_invariant ? 0 : resident_workgroups(k_gemm_f32, 256), 4);
}

int tune_expand_f32(bh_plan* p, int64_t B, hipStream_t s) {
  const int64_t M_pad = ((B + BM - 1) / BM) * BM;
  const int64_t mt = M_pad / BM, nt = p->C_pad / BN;
  const int64_t nk_total = p->VR_pad / BK;
  const size_t fbytes = (size_t)kParityClasses * p->VR_pad * M_pad * sizeof(float);
  int rc;
  if ((rc = grow(p->gathered, fbytes)) != BH_OK) return rc;
  if ((rc = grow(p->partial, (size_t)16 * M_pad * p->C_pad * sizeof(float))) != BH_OK) return rc;
  float* Ft = (float*)p->gathered.ptr;
  float* part = (float*)p->partial.ptr;
  BH_HIP(hipMemsetAsync(Ft, 0, fbytes, s));   // timing data: any finite values
  float best_ms = 1e30f;
  int best = 1;
  for (int ns = 1; ns <= kMaxSplit; ++ns) {
    if (ns > 1 && nk_total / ns < 8) break;
    float ms = 0.0f;
    rc = time_on_stream(
        s, 2, [] {},
        [&] {
          hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)(mt * nt * ns)), dim3(256), 0, s, Ft,
                             p->psi, part, M_pad, p->C_pad, p->VR_pad, p->ctiles, nk_total, ns);
        },
        &ms);
    if (rc != BH_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best = ns;
    }
  }
  p->tuned_split[0][mt] = best;
  return BH_OK;
}

}  // namespace bh
