// Expansion on BF16 MFMA with FP32 accumulation (Sec. II-A, the coefficients
// a = h^3 Psi^T f), and its split-BF16 refinement.
//
// Every FP32 value x is split as x = hi + lo + r with hi = bf16(x),
// lo = bf16(x - hi), |r| <= 2^-16 |x| or so.  Then
//   coarse  = Psi_hi^T F_hi                      (relative error ~ 2^-8)
//   refined = coarse + Psi_hi^T F_lo + Psi_lo^T F_hi   (~ 2^-16: FP32-level)
// Both are computed by one kernel with two accumulator sets; the three
// products use v_mfma_f32_32x32x16_bf16.
//
//   k_psi_split : Psi[VR_pad][C_pad] FP32 -> Ph, Pl [C_pad][VR_pad] BF16 (once per plan)
//   k_gather_split: vols -> Fh, Fl [8][M_pad][VR_pad] BF16: the mirror sums
//                 of each parity class at the orbit representatives (as the
//                 FP32 path), zero padded
//   k_gemm_bf16 : split-K partial sums, 128x128 tiles, K step 32 voxels; a
//                 column tile reads the slice of its class
//   k_reduce2   : sums splits, scatters to the complex layout
//
// Operands are K-contiguous rows (particles, coefficients), copied into LDS
// by LDS-DMA loads with the 16-byte chunks of each row XOR-swizzled so that
// fragment reads of eight consecutive rows fall in distinct banks.  A lane's
// fragment is eight consecutive voxels of one row; the same voxel-to-lane map
// is used for both operands, so the sum over voxels is exact whatever order
// the instruction takes it in.
#include "bh_internal.h"

#include <algorithm>

namespace bh {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, BK = 32;

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ inline uint16_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Ph[c][v], Pl[c][v] from Psi[v][c]: 32x32 LDS transpose and split.
__global__ __launch_bounds__(256) void k_psi_split(const float* __restrict__ psi, int64_t VR_pad,
                                                   int64_t C_pad, uint16_t* __restrict__ ph,
                                                   uint16_t* __restrict__ pl) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t v0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
#pragma unroll
  for (int i = 0; i < 4; ++i) tile[ty + 8 * i][tx] = psi[(v0 + ty + 8 * i) * C_pad + c0 + tx];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float x = tile[tx][ty + 8 * i];
    const uint16_t h = bf16_bits(x);
    const int64_t o = (c0 + ty + 8 * i) * VR_pad + v0 + tx;
    ph[o] = h;
    pl[o] = bf16_bits(x - bf16_value(h));
  }
}

// Fh[P][b][v], Fl[P][b][v] = split of the class-P mirror sum of particle b
// at representative v (0 outside v < VR, b < B).  Particle b's volume is
// vols[rows[b]] with a row table (a row outside [0, n_rows) reads as NaN
// and raises the error word `bad`), else vols[b].
__global__ __launch_bounds__(256) void k_gather_split(const float* __restrict__ vols,
                                                      int64_t vol_stride, int64_t B,
                                                      const int64_t* __restrict__ rows,
                                                      int64_t n_rows, int* bad,
                                                      const int32_t* __restrict__ vrep, int64_t VR,
                                                      int64_t VR_pad, int64_t M_pad, int N,
                                                      uint16_t* __restrict__ fh,
                                                      uint16_t* __restrict__ fl) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= VR_pad) return;
  int32_t off[8];
  mirror_offsets((v < VR) ? vrep[v] : 0, N, off);
  const int64_t slab = M_pad * VR_pad;
  for (int64_t b = blockIdx.y; b < M_pad; b += gridDim.y) {
    float f[8];
    const int64_t r = volume_row(rows, n_rows, B, b, v == 0 ? bad : nullptr);
    const bool in = v < VR && r >= 0;
    const float* vb = vols + (in ? r * vol_stride : 0);
    const float outside = r == -2 ? __builtin_nanf("") : 0.0f;
#pragma unroll
    for (int s = 0; s < 8; ++s) f[s] = in ? vb[off[s]] : outside;
    parity_fold(f);
#pragma unroll
    for (int c = 0; c < kParityClasses; ++c) {
      const uint16_t h = bf16_bits(f[c]);
      fh[c * slab + b * VR_pad + v] = h;
      fl[c * slab + b * VR_pad + v] = bf16_bits(f[c] - bf16_value(h));
    }
  }
}

typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

// LDS of one K step: the 128 rows of Fh, Ph (and Fl, Pl with the
// correction), 64 bytes each (four 16-byte chunks); two steps alternate.
constexpr int kRowBytes = BK * 2, kArrBytes = BM * kRowBytes;   // BM == BN
template <bool LO>
struct StepLds {
  static constexpr int ah = 0, bh = kArrBytes, al = 2 * kArrBytes, bl = 3 * kArrBytes;
  static constexpr int bytes = (LO ? 4 : 2) * kArrBytes;
};

// Chunk c of row r sits at chunk position c ^ g(r), g(r) = (r1 ^ r3) + 2 r2
// for the bits r1..r3 of r: the 16-byte fragment reads of any eight
// consecutive rows fall in distinct 16-byte bank groups of a 128-byte span,
// and those of any sixteen in distinct ones of a 256-byte span (rows are
// 64 bytes, so rows r and r + 4 share banks).  The previous g(r) = r1 + 2 r2
// gave sixteen rows two-way conflicts (measured: bank-conflict cycles four
// times the LDS instruction cycles).
__device__ inline int step_swz(int c, int r) {
  return c ^ ((((r >> 1) ^ (r >> 3)) & 1) | (((r >> 2) & 1) << 1));
}

// Wait for this wave's LDS reads and LDS-DMA loads, then the barrier.
// (Written out: the compiler's barrier adds nothing here, and its own wait
// placement does not know about the DMA loads.)
__device__ inline void dma_barrier() {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// COARSE: part_c += Fh Ph^T.  CORR: part_r += Fh Pl^T + Fl Ph^T.
//
// 4 waves in a 2 x 2 arrangement, each 64 x 64 as 2 x 2 MFMA tiles per
// accumulator set.  The operands of K step kt + 1 are copied global -> LDS
// by the waves' LDS-DMA loads (16 bytes per lane straight into LDS; a load
// covers 16 rows of one array, lane i -> LDS bytes 16 i, the lane fetching
// the chunk the swizzle places there) while step kt is computed; no
// register staging, so the fragments of both 16-voxel halves of a step can
// be read before its MFMAs run.  Only `smem` lives in LDS: with a second LDS
// variable the compiler would wait for every DMA load before each read.
template <bool COARSE, bool CORR>
__global__ __launch_bounds__(256, 2) void k_gemm_bf16(const uint16_t* __restrict__ fh,
                                                      const uint16_t* __restrict__ fl,
                                                      const uint16_t* __restrict__ ph,
                                                      const uint16_t* __restrict__ pl,
                                                      float* __restrict__ part_c,
                                                      float* __restrict__ part_r, int64_t M_pad,
                                                      int64_t C_pad, int64_t VR_pad, ClassTiles ct,
                                                      int64_t nk_total, int nsplit) {
  constexpr bool LO = CORR;
  using St = StepLds<LO>;
  __shared__ __attribute__((aligned(1024))) char smem[2 * St::bytes];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int64_t tm, tn, ts;
  gemm_tile(blockIdx.x, M_pad / BM, C_pad / BN, nsplit, tm, tn, ts);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  int64_t k0, nk64;
  split_range(ts, nsplit, nk_total, k0, nk64);
  const int nk = (int)nk64;
  const int64_t k_begin = k0 * BK;
  const int64_t slab = class_of_tile(ct, tn) * M_pad * VR_pad;
  // DMA: wave w loads rows 32 w .. 32 w + 31 of each array as two blocks of
  // 16 rows; lane -> row 32 w + lane / 4 (+ 16), stored chunk lane % 4
  const int lrow = 32 * wave + (lane >> 2);
  const int lchunk = step_swz(lane & 3, lrow);
  const uint16_t* ga_h = fh + slab + (m0 + lrow) * VR_pad + k_begin + 8 * lchunk;
  const uint16_t* gb_h = ph + (n0 + lrow) * VR_pad + k_begin + 8 * lchunk;
  const uint16_t* ga_l = LO ? fl + slab + (m0 + lrow) * VR_pad + k_begin + 8 * lchunk : nullptr;
  const uint16_t* gb_l = LO ? pl + (n0 + lrow) * VR_pad + k_begin + 8 * lchunk : nullptr;
  const int64_t next16 = 16 * VR_pad;
  const int dst = wave * 2048;
  auto issue = [&](int kt) {
    char* st = smem + (kt & 1) * St::bytes + dst;
    const int64_t ko = (int64_t)kt * BK;
    __builtin_amdgcn_global_load_lds((global_void*)(ga_h + ko), (lds_void*)(st + St::ah), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((global_void*)(ga_h + next16 + ko), (lds_void*)(st + St::ah + 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((global_void*)(gb_h + ko), (lds_void*)(st + St::bh), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((global_void*)(gb_h + next16 + ko), (lds_void*)(st + St::bh + 1024), 16, 0, 0);
    if (LO) {
      __builtin_amdgcn_global_load_lds((global_void*)(ga_l + ko), (lds_void*)(st + St::al), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((global_void*)(ga_l + next16 + ko), (lds_void*)(st + St::al + 1024), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((global_void*)(gb_l + ko), (lds_void*)(st + St::bl), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((global_void*)(gb_l + next16 + ko), (lds_void*)(st + St::bl + 1024), 16, 0, 0);
    }
  };
  floatx16 c00 = {}, c01 = {}, c10 = {}, c11 = {};
  floatx16 d00 = {}, d01 = {}, d10 = {}, d11 = {};
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int hl = lane >> 5, ll = lane & 31;
  // fragment rows wm + ll, wm + 32 + ll (A), wn + ll, wn + 32 + ll (B): the
  // swizzle depends on ll only (wm, wn are multiples of 64)
  const int fa0 = (wm + ll) * kRowBytes, fa1 = fa0 + 32 * kRowBytes;
  const int fb0 = (wn + ll) * kRowBytes, fb1 = fb0 + 32 * kRowBytes;
  issue(0);
  for (int kt = 0; kt < nk; ++kt) {
    dma_barrier();                   // step kt landed; step kt - 1's buffer is free
    if (kt + 1 < nk) issue(kt + 1);
    const char* st = smem + (kt & 1) * St::bytes;
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int co = 16 * step_swz(2 * ks + hl, ll);
      auto frag = [&](int off) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(st + off + co));
      };
      const bf16x8 ah0 = frag(St::ah + fa0), ah1 = frag(St::ah + fa1);
      const bf16x8 bh0 = frag(St::bh + fb0), bh1 = frag(St::bh + fb1);
      if (COARSE) {
        c00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bh0, c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bh1, c01, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bh0, c10, 0, 0, 0);
        c11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bh1, c11, 0, 0, 0);
      }
      if (CORR) {
        const bf16x8 al0 = frag(St::al + fa0), al1 = frag(St::al + fa1);
        const bf16x8 bl0 = frag(St::bl + fb0), bl1 = frag(St::bl + fb1);
        d00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bl0, d00, 0, 0, 0);
        d01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, bl1, d01, 0, 0, 0);
        d10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bl0, d10, 0, 0, 0);
        d11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah1, bl1, d11, 0, 0, 0);
        d00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, bh0, d00, 0, 0, 0);
        d01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, bh1, d01, 0, 0, 0);
        d10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, bh0, d10, 0, 0, 0);
        d11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al1, bh1, d11, 0, 0, 0);
      }
    }
  }
  const int64_t row0 = m0 + wm + 4 * hl, col0 = n0 + wn + ll;
  float* oc = part_c + ts * M_pad * C_pad;
  float* orr = part_r + ts * M_pad * C_pad;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = row0 + 8 * (r >> 2) + (r & 3);
    if (COARSE) {
      oc[row * C_pad + col0] = c00[r];
      oc[row * C_pad + col0 + 32] = c01[r];
      oc[(row + 32) * C_pad + col0] = c10[r];
      oc[(row + 32) * C_pad + col0 + 32] = c11[r];
    }
    if (CORR) {
      orr[row * C_pad + col0] = d00[r];
      orr[row * C_pad + col0 + 32] = d01[r];
      orr[(row + 32) * C_pad + col0] = d10[r];
      orr[(row + 32) * C_pad + col0 + 32] = d11[r];
    }
  }
}

// coeffs = sum_s (coarse + corr) (corr absent: coarse only); coarse_out = sum_s coarse.
__global__ __launch_bounds__(256) void k_reduce2(const float* __restrict__ part_c,
                                                 const float* __restrict__ part_r, int nsplit,
                                                 int64_t M_pad, int64_t C_pad, int64_t B, int64_t C,
                                                 const int32_t* __restrict__ csrc,
                                                 const float* __restrict__ csgn,
                                                 float* __restrict__ coeffs,
                                                 float* __restrict__ coarse_out, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * C) return;
  const int64_t b = t / C, q = t % C;
  const int32_t sr = csrc[2 * q], si = csrc[2 * q + 1];
  // every split's loads first (in flight together), then the sums in split order
  float vcr[kMaxSplit], vci[kMaxSplit], vrr[kMaxSplit], vri[kMaxSplit];
#pragma unroll
  for (int s = 0; s < kMaxSplit; ++s) {
    if (s < nsplit) {
      const int64_t o = (int64_t)s * M_pad * C_pad + b * C_pad;
      vcr[s] = part_c[o + sr];
      vci[s] = si >= 0 ? part_c[o + si] : 0.0f;
      vrr[s] = part_r ? part_r[o + sr] : 0.0f;
      vri[s] = (part_r && si >= 0) ? part_r[o + si] : 0.0f;
    }
  }
  float cre = 0.0f, cim = 0.0f, rre = 0.0f, rim = 0.0f;
#pragma unroll
  for (int s = 0; s < kMaxSplit; ++s) {
    if (s < nsplit) {
      cre += vcr[s];
      cim += vci[s];
      rre += vrr[s];
      rim += vri[s];
    }
  }
  const float gr = csgn[2 * q], gi = csgn[2 * q + 1];
  const int64_t oc = b * ldc + q;
  coeffs[2 * oc] = (cre + rre) * gr;
  coeffs[2 * oc + 1] = (si >= 0) ? (cim + rim) * gi : 0.0f;
  if (coarse_out) {
    coarse_out[2 * oc] = cre * gr;
    coarse_out[2 * oc + 1] = (si >= 0) ? cim * gi : 0.0f;
  }
}

}  // namespace

int ensure_bf16_basis(bh_plan* p) {
  if (p->psi_h) return BH_OK;
  const size_t n = (size_t)p->C_pad * p->VR_pad;
  if (hipMalloc((void**)&p->psi_h, n * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc((void**)&p->psi_l, n * sizeof(uint16_t)) != hipSuccess) {
    if (p->psi_h) (void)hipFree(p->psi_h);
    p->psi_h = nullptr;
    p->psi_l = nullptr;
    (void)hipGetLastError();
    return set_error(BH_ENOMEM, "BF16 basis allocation failed");
  }
  hipLaunchKernelGGL(k_psi_split, dim3((unsigned)(p->VR_pad / 32), (unsigned)(p->C_pad / 32)),
                     dim3(256), 0, 0, p->psi, p->VR_pad, p->C_pad, p->psi_h, p->psi_l);
  BH_HIP(hipGetLastError());
  BH_HIP(hipDeviceSynchronize());
  return BH_OK;
}

int launch_expand_bf16(bh_plan* p, const float* vols, int64_t B, bool refine, float* coeffs,
                       float* coarse_out, hipStream_t s, bool batch_invariant, int64_t ldc,
                       const int64_t* rows, int64_t n_rows) {
  if (ldc <= 0) ldc = p->C;
  if (B == 0) return BH_OK;
  int rc = ensure_bf16_basis(p);
  if (rc != BH_OK) return rc;
  const int64_t M_pad = ((B + BM - 1) / BM) * BM;
  const int64_t mt = M_pad / BM, nt = p->C_pad / BN;
  const int64_t nk_total = p->VR_pad / BK;   // multiple of 16
  const int nsplit = expand_split_bf16(p, B, batch_invariant, refine);
  const size_t fbytes = (size_t)kParityClasses * M_pad * p->VR_pad * sizeof(uint16_t);
  const size_t pbytes = (size_t)nsplit * M_pad * p->C_pad * sizeof(float);
  if ((rc = grow(p->gathered, 2 * fbytes)) != BH_OK) return rc;
  if ((rc = grow(p->partial, (refine ? 2 : 1) * pbytes)) != BH_OK) return rc;
  uint16_t* fh = (uint16_t*)p->gathered.ptr;
  uint16_t* fl = fh + fbytes / sizeof(uint16_t);
  float* part_c = (float*)p->partial.ptr;
  float* part_r = refine ? part_c + (size_t)nsplit * M_pad * p->C_pad : nullptr;
  const int64_t vol_stride = (int64_t)p->N * p->N * p->N;
  {
    ProfScope ps(p, "gather_bf16", s, B);
    const unsigned gy = (unsigned)(M_pad < 4096 ? M_pad : 4096);
    hipLaunchKernelGGL(k_gather_split, dim3((unsigned)((p->VR_pad + 255) / 256), gy), dim3(256),
                       0, s, vols, vol_stride, B, rows, n_rows, p->err_dev, p->vrep, p->VR,
                       p->VR_pad, M_pad, p->N, fh, fl);
  }
  BH_HIP(hipGetLastError());
  {
    ProfScope ps(p, refine ? "gemm_bf16x3" : "gemm_bf16", s, B);
    const dim3 grid((unsigned)(mt * nt * nsplit));
    if (refine)
      hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, dim3(256), 0, s, fh, fl, p->psi_h,
                         p->psi_l, part_c, part_r, M_pad, p->C_pad, p->VR_pad, p->ctiles,
                         nk_total, nsplit);
    else
      hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, s, fh, fl, p->psi_h,
                         p->psi_l, part_c, part_c, M_pad, p->C_pad, p->VR_pad, p->ctiles,
                         nk_total, nsplit);
  }
  BH_HIP(hipGetLastError());
  {
    ProfScope ps(p, "reduce", s, B);
    const int64_t tot = B * p->C;
    hipLaunchKernelGGL(k_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part_c,
                       part_r, nsplit, M_pad, p->C_pad, B, p->C, p->csrc, p->csgn, coeffs,
                       coarse_out, ldc);
  }
  BH_HIP(hipGetLastError());
  return BH_OK;
}

// q = 18: a tile's 128 KB of coarse and corrected partial sums, written and
// read back, against the chip-wide time of a K-step (about 1.5 us per
// workgroup); 9 for the coarse sums alone.
int expand_split_bf16(const bh_plan* p, int64_t B, bool batch_invariant, bool refine) {
  const int64_t mt = (B + BM - 1) / BM, nt = p->C_pad / BN, nk_total = p->VR_pad / BK;
  int64_t slots = 0;
  if (!batch_invariant)
    slots = refine ? resident_workgroups(k_gemm_bf16<true, true>, 256)
                   : resident_workgroups(k_gemm_bf16<true, false>, 256);
  return expand_split(mt, nt, nk_total, batch_invariant, &p->tuned_split[1], slots,
                      refine ? 18 : 9);
}

int tune_expand_bf16(bh_plan* p, int64_t B, hipStream_t s) {
  int rc = ensure_bf16_basis(p);
  if (rc != BH_OK) return rc;
  const int64_t M_pad = ((B + BM - 1) / BM) * BM;
  const int64_t mt = M_pad / BM, nt = p->C_pad / BN;
  const int64_t nk_total = p->VR_pad / BK;
  const size_t fbytes = (size_t)kParityClasses * M_pad * p->VR_pad * sizeof(uint16_t);
  if ((rc = grow(p->gathered, 2 * fbytes)) != BH_OK) return rc;
  if ((rc = grow(p->partial, (size_t)2 * 16 * M_pad * p->C_pad * sizeof(float))) != BH_OK)
    return rc;
  uint16_t* fh = (uint16_t*)p->gathered.ptr;
  uint16_t* fl = fh + fbytes / sizeof(uint16_t);
  float* part = (float*)p->partial.ptr;
  BH_HIP(hipMemsetAsync(fh, 0, 2 * fbytes, s));   // timing data: any finite values
  float best_ms = 1e30f;
  int best = 1;
  for (int ns = 1; ns <= kMaxSplit; ++ns) {
    if (ns > 1 && nk_total / ns < 8) break;
    float ms = 0.0f;
    rc = time_on_stream(
        s, 2, [] {},
        [&] {
          hipLaunchKernelGGL((k_gemm_bf16<true, true>), dim3((unsigned)(mt * nt * ns)), dim3(256),
                             0, s, fh, fl, p->psi_h, p->psi_l, part,
                             part + (size_t)ns * M_pad * p->C_pad, M_pad, p->C_pad, p->VR_pad,
                             p->ctiles, nk_total, ns);
        },
        &ms);
    if (rc != BH_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best = ns;
    }
  }
  p->tuned_split[1][mt] = best;
  return BH_OK;
}

}  // namespace bh
