// Point kernels of the kiFMM on gfx950: charge gather into Morton order,
// P2M check potentials (Section 2.1.1) and the fused leaf evaluation
// L2P + P2P (Section 2, downward pass).  Laplace kernel 1 / (4 pi r), zero
// at r = 0 (pairs with r^2 below the smallest normal number of the working
// precision count as coincident).
#include <algorithm>

#include "group.h"
#include "kernels.h"

namespace kifmm {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;

// 1 / sqrt(r2), branch-free.  FP64: the hardware estimate y refined by one
// third-order step of the series (1 - e)^(-1/2) = 1 + e/2 + 3 e^2/8 + ...
// with e = 1 - r2 y^2, which cubes the estimate's relative error.  FP32:
// the hardware result as is (about 1 ulp).
__device__ inline double inv_r(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2 * y, y, 1.0);
  const double r = fma(y * e, fma(e, 0.375, 0.5), y);
  return r2 >= 2.2250738585072014e-308 ? r : 0.0;
}
__device__ inline float inv_r(float r2) {
  const float r = __builtin_amdgcn_rsqf(r2);
  return r2 >= 1.17549435e-38f ? r : 0.0f;
}

template <typename TQ>
__global__ void gather_kernel(const TQ* __restrict__ q, int64_t ldq, const int64_t* __restrict__ perm,
                              int64_t n, TQ* __restrict__ qs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (i < n) qs[v * n + i] = q[v * ldq + perm[i]];
}

// Grouped gather: a job's workgroups are (x, v) with x fastest, ceil(n / 256)
// per vector.
template <typename TQ>
__global__ void gather_group_kernel(const GatherArgs* __restrict__ jobs, const int64_t* __restrict__ pre,
                                    int nj) {
  int64_t b;
  const GatherArgs a = jobs[group_job(pre, nj, b)];
  const int64_t nbx = (a.n + 255) / 256;
  const int64_t v = b / nbx;
  const int64_t i = (b - v * nbx) * 256 + threadIdx.x;
  const TQ* __restrict__ q = static_cast<const TQ*>(a.q);
  TQ* __restrict__ qs = static_cast<TQ*>(a.qs);
  if (i < a.n) qs[v * a.n + i] = q[v * a.ldq + a.perm[i]];
}

constexpr int kP2MChunk = 64;  // sources staged per pass (one per lane)

// One wave per leaf.  Each lane owns PPL upward-check points (lane + 64 j)
// and NV charge vectors, so one staged source (x, y, z, q) serves PPL x NV
// accumulations; the source loop is uniform across the wave.
template <typename TQ, int PPL, int NV>
__device__ __forceinline__ void p2m_body(const P2MArgs& a, int64_t leaf) {
  const double* __restrict__ xyz = a.xyz;
  const TQ* __restrict__ qs = static_cast<const TQ*>(a.qs);
  const int64_t n_src = a.n_src;
  const int32_t* __restrict__ start = a.start;
  const int32_t* __restrict__ end = a.end;
  const double* __restrict__ centers = a.centers;
  const double* __restrict__ surf = a.surf;
  const double ar = a.ar;
  const int ns = a.ns, nvec = a.nvec;
  double* __restrict__ phi = a.phi;
  constexpr int NX = NV > 1 ? NV - 1 : 1;
  __shared__ double4 sp[kP2MChunk];
  __shared__ double sq[NX][kP2MChunk];
  const int lane = threadIdx.x;
  const int s0 = start[leaf], s1 = end[leaf];
  const double cx = centers[3 * leaf], cy = centers[3 * leaf + 1], cz = centers[3 * leaf + 2];
  for (int i0 = 0; i0 < ns; i0 += 64 * PPL) {
    double px[PPL], py[PPL], pz[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int i = min(i0 + lane + 64 * j, ns - 1);  // surplus lanes repeat a point, unwritten
      px[j] = cx + ar * surf[3 * i];
      py[j] = cy + ar * surf[3 * i + 1];
      pz[j] = cz + ar * surf[3 * i + 2];
    }
    for (int vb = 0; vb < nvec; vb += NV) {
      double acc[PPL][NV];
#pragma unroll
      for (int j = 0; j < PPL; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[j][v] = 0.0;
      for (int c0 = s0; c0 < s1; c0 += kP2MChunk) {
        const int cn = min(kP2MChunk, s1 - c0);
        __syncthreads();
        if (lane < cn) {
          const int64_t si = c0 + lane;
          sp[lane] = double4{xyz[3 * si], xyz[3 * si + 1], xyz[3 * si + 2],
                             (double)qs[(int64_t)vb * n_src + si]};
#pragma unroll
          for (int v = 1; v < NV; ++v)
            sq[v - 1][lane] = vb + v < nvec ? (double)qs[(int64_t)(vb + v) * n_src + si] : 0.0;
        }
        __syncthreads();
        for (int s = 0; s < cn; ++s) {
          const double4 src = sp[s];
#pragma unroll
          for (int j = 0; j < PPL; ++j) {
            const double dx = px[j] - src.x, dy = py[j] - src.y, dz = pz[j] - src.z;
            const double ir = inv_r(dx * dx + dy * dy + dz * dz);
            acc[j][0] += ir * src.w;
#pragma unroll
            for (int v = 1; v < NV; ++v) acc[j][v] += ir * sq[v - 1][s];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const int i = i0 + lane + 64 * j;
        if (i >= ns) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (vb + v < nvec) phi[((int64_t)leaf * nvec + vb + v) * ns + i] = kInv4Pi * acc[j][v];
      }
    }
  }
}

template <typename TQ, int PPL, int NV>
__global__ __launch_bounds__(64) void p2m_kernel(P2MArgs a) {
  p2m_body<TQ, PPL, NV>(a, blockIdx.x);
}

template <typename TQ, int PPL, int NV>
__global__ __launch_bounds__(64) void p2m_group_kernel(const P2MArgs* __restrict__ jobs,
                                                       const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const P2MArgs a = jobs[group_job(pre, nj, b)];
  p2m_body<TQ, PPL, NV>(a, b);
}

// Instance of the P2M kernel: (TQ, check points per lane, vector block).
int p2m_instance(bool q_fp64, int ns, int nvec) {
  const int ppl = std::min(4, (ns + 63) / 64);
  const int nv = nvec == 1 ? 0 : nvec == 2 ? 1 : nvec <= 4 ? 2 : 3;
  return (q_fp64 ? 16 : 0) + (ppl - 1) * 4 + nv;
}

// One launch of instance `inst`: a plain launch of one job (jobs == nullptr,
// `one` holds the arguments) or a grouped launch.
template <typename TQ, int PPL, int NV>
void p2m_go(const P2MArgs* one, const P2MArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
            hipStream_t s) {
  if (!jobs)
    p2m_kernel<TQ, PPL, NV><<<(unsigned)blocks, 64, 0, s>>>(*one);
  else
    p2m_group_kernel<TQ, PPL, NV><<<(unsigned)blocks, 64, 0, s>>>(jobs, pre, nj);
}

template <typename TQ, int PPL>
void p2m_go_nv(int nv, const P2MArgs* one, const P2MArgs* jobs, const int64_t* pre, int nj,
               int64_t blocks, hipStream_t s) {
  if (nv == 0) p2m_go<TQ, PPL, 1>(one, jobs, pre, nj, blocks, s);
  else if (nv == 1) p2m_go<TQ, PPL, 2>(one, jobs, pre, nj, blocks, s);
  else if (nv == 2) p2m_go<TQ, PPL, 4>(one, jobs, pre, nj, blocks, s);
  else p2m_go<TQ, PPL, 8>(one, jobs, pre, nj, blocks, s);
}

template <typename TQ>
void p2m_go_ppl(int ppl, int nv, const P2MArgs* one, const P2MArgs* jobs, const int64_t* pre, int nj,
                int64_t blocks, hipStream_t s) {
  if (ppl == 1) p2m_go_nv<TQ, 1>(nv, one, jobs, pre, nj, blocks, s);
  else if (ppl == 2) p2m_go_nv<TQ, 2>(nv, one, jobs, pre, nj, blocks, s);
  else if (ppl == 3) p2m_go_nv<TQ, 3>(nv, one, jobs, pre, nj, blocks, s);
  else p2m_go_nv<TQ, 4>(nv, one, jobs, pre, nj, blocks, s);
}

hipError_t p2m_dispatch(int inst, const P2MArgs* one, const P2MArgs* jobs, const int64_t* pre, int nj,
                        int64_t blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (inst < 0 || inst >= 32 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int ppl = (inst % 16) / 4 + 1, nv = inst % 4;
  if (inst >= 16)
    p2m_go_ppl<double>(ppl, nv, one, jobs, pre, nj, blocks, s);
  else
    p2m_go_ppl<float>(ppl, nv, one, jobs, pre, nj, blocks, s);
  return hipGetLastError();
}

constexpr int kLeafThreads = 128;
constexpr int kLeafChunk = 256;  // near-field sources staged per pass (multiple of 16)
constexpr int kL2PChunk = 160;   // downward-equivalent points staged per pass (multiple of 16)

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// One workgroup per target leaf.  Sources are staged in LDS as (x, y, z, q)
// quadruples (further charge vectors in separate arrays), so one LDS read
// serves an interaction; each thread owns two targets, so each staged
// source is used twice; 1 to 8 lanes share a target pair (by leaf
// occupancy), split the staged sources and reduce with cross-lane shuffles.
// The near-field sources (up to 27 leaves, each a contiguous run in Morton
// order) are located by binary search over the run offsets.  L2P runs in
// FP64 from the leaf's downward-equivalent densities; P2P runs in T, in the
// frame of the target leaf's center (offsets of at most 1.5 leaf widths w,
// formed in FP64).  In FP32 each offset is split as hi + lo (hi its FP32
// rounding, lo the FP32 rounding of the remainder); pairs are evaluated
// from the hi parts, whose rounding (at most about 1e-7 w) bounds the
// relative error of r by 5e-6 for r >= w / 16.  The rare pairs closer than
// that (r^2 < tau2) are evaluated again from the difference of the hi
// parts plus the difference of the lo parts, which carries the pair's
// separation to FP32 relative accuracy.  NV
// charge vectors are handled per pass.  MODE 0 does both; MODE 1 only the
// near field, storing its raw sums (in T, before the 1/(4 pi) factor);
// MODE 2 adds the far field to those stored sums and finishes, so 1 then 2
// gives exactly the result of 0.
template <typename T, typename TQ, int NV, int MODE>
__device__ __forceinline__ void leaf_eval_body(const LeafArgs& a, int64_t blk) {
  const double* __restrict__ txyz = a.txyz;
  const double* __restrict__ sxyz = a.sxyz;
  const TQ* __restrict__ qs = static_cast<const TQ*>(a.qs);
  const int64_t n_src = a.n_src;
  const int32_t* __restrict__ tstart = a.tstart;
  const int32_t* __restrict__ tend = a.tend;
  const int32_t* __restrict__ sstart = a.sstart;
  const int32_t* __restrict__ send = a.send;
  const int64_t* __restrict__ noffs = a.near_offs;
  const int32_t* __restrict__ nsrc = a.near_src;
  const double* __restrict__ centers = a.centers;
  const double* __restrict__ surf = a.surf;
  const double ar = a.ar;
  const int ns = a.ns;
  const double* __restrict__ local = a.local;
  const int64_t* __restrict__ tperm = a.tgt_perm;
  TQ* __restrict__ phi = static_cast<TQ*>(a.phi);
  const int64_t ldphi = a.ldphi;
  const int nvec = a.nvec;
  const int64_t n_leaf = a.n_leaf;
  const T tau2 = (T)a.tau2;
  using T4 = typename Vec4<T>::type;
  constexpr int NX = NV > 1 ? NV - 1 : 1;
  __shared__ double4 ls[kL2PChunk];
  __shared__ double lq[NX][kL2PChunk];
  constexpr bool kSplit = sizeof(T) == 4;  // FP32: hi + lo offsets
  __shared__ T4 ps[kLeafChunk];
  __shared__ float4 pl[kSplit ? kLeafChunk : 1];  // lo parts of the staged offsets
  __shared__ T pq[NX][kLeafChunk];
  __shared__ int32_t nb_first[27];
  __shared__ int32_t nb_pref[28];
  __shared__ int32_t n_nb;

  // consecutive leaves (which share most near-field sources) on one XCD;
  // the grid is 8 ceil(n_leaf / 8) workgroups
  const int64_t per_xcd = (n_leaf + 7) / 8;
  const int64_t leaf = (blk % 8) * per_xcd + blk / 8;
  if (leaf >= n_leaf) return;
  const int t0 = tstart[leaf], t1 = tend[leaf];
  const int nt = t1 - t0;
  if (nt == 0) return;
  if (threadIdx.x == 0) {
    const int64_t a = noffs[leaf], b = noffs[leaf + 1];
    int acc = 0;
    int k = 0;
    for (int64_t e = a; e < b && k < 27; ++e, ++k) {
      const int32_t s = nsrc[e];
      nb_first[k] = sstart[s];
      nb_pref[k] = acc;
      acc += send[s] - sstart[s];
    }
    nb_pref[k] = acc;
    n_nb = k;
  }
  __syncthreads();
  const int nnb = n_nb;
  const int total = nb_pref[nnb];
  const int pairs = (nt + 1) / 2;
  const int L = pairs <= 16 ? 8 : pairs <= 32 ? 4 : pairs <= 64 ? 2 : 1;
  const int slots = kLeafThreads / L;
  const int tp = threadIdx.x / L, sub = threadIdx.x % L;
  const double cx = centers[3 * leaf], cy = centers[3 * leaf + 1], cz = centers[3 * leaf + 2];

  for (int vb = 0; vb < nvec; vb += NV) {
    for (int pb = 0; pb < pairs; pb += slots) {
      const int ti0 = 2 * (pb + tp), ti1 = ti0 + 1;
      const bool act0 = ti0 < nt, act1 = ti1 < nt;
      double x0 = 0, y0 = 0, z0 = 0, x1 = 0, y1 = 0, z1 = 0;
      if (act0) {
        x0 = txyz[3 * (int64_t)(t0 + ti0)];
        y0 = txyz[3 * (int64_t)(t0 + ti0) + 1];
        z0 = txyz[3 * (int64_t)(t0 + ti0) + 2];
      }
      if (act1) {
        x1 = txyz[3 * (int64_t)(t0 + ti1)];
        y1 = txyz[3 * (int64_t)(t0 + ti1) + 1];
        z1 = txyz[3 * (int64_t)(t0 + ti1) + 2];
      }
      double al0[NV], al1[NV];
      T ap0[NV], ap1[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        al0[v] = al1[v] = 0.0;
        ap0[v] = ap1[v] = T(0);
      }
      // L2P: the leaf's downward-equivalent surface as sources (FP64)
      for (int c0 = 0; c0 < (MODE == 1 ? 0 : ns); c0 += kL2PChunk) {
        const int cn = min(kL2PChunk, ns - c0);
        const int cnp = (cn + 2 * L - 1) / (2 * L) * (2 * L);  // zero densities pad
        __syncthreads();
        for (int t = threadIdx.x; t < cnp; t += kLeafThreads) {
          if (t < cn) {
            ls[t] = double4{cx + ar * surf[3 * (c0 + t)], cy + ar * surf[3 * (c0 + t) + 1],
                            cz + ar * surf[3 * (c0 + t) + 2],
                            local[((int64_t)leaf * nvec + vb) * ns + c0 + t]};
#pragma unroll
            for (int v = 1; v < NV; ++v)
              lq[v - 1][t] = vb + v < nvec ? local[((int64_t)leaf * nvec + vb + v) * ns + c0 + t] : 0.0;
          } else {
            ls[t] = double4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int v = 1; v < NV; ++v) lq[v - 1][t] = 0.0;
          }
        }
        __syncthreads();
        auto l2p = [&](int s) {
          const double4 src = ls[s];
          const double dx0 = x0 - src.x, dy0 = y0 - src.y, dz0 = z0 - src.z;
          const double dx1 = x1 - src.x, dy1 = y1 - src.y, dz1 = z1 - src.z;
          const double r0 = inv_r(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
          const double r1 = inv_r(dx1 * dx1 + dy1 * dy1 + dz1 * dz1);
          al0[0] += r0 * src.w;
          al1[0] += r1 * src.w;
#pragma unroll
          for (int v = 1; v < NV; ++v) {
            const double qv = lq[v - 1][s];
            al0[v] += r0 * qv;
            al1[v] += r1 * qv;
          }
        };
        for (int s0 = 0; s0 < cnp; s0 += 2 * L) {
          l2p(s0 + sub);
          l2p(s0 + L + sub);
        }
      }
      // P2P over the near field
      const T xt0 = (T)(x0 - cx), yt0 = (T)(y0 - cy), zt0 = (T)(z0 - cz);
      const T xt1 = (T)(x1 - cx), yt1 = (T)(y1 - cy), zt1 = (T)(z1 - cz);
      const float xl0 = (float)((x0 - cx) - (double)xt0), yl0 = (float)((y0 - cy) - (double)yt0),
                  zl0 = (float)((z0 - cz) - (double)zt0);
      const float xl1 = (float)((x1 - cx) - (double)xt1), yl1 = (float)((y1 - cy) - (double)yt1),
                  zl1 = (float)((z1 - cz) - (double)zt1);
      for (int c0 = 0; c0 < (MODE == 2 ? 0 : total); c0 += kLeafChunk) {
        const int cn = min(kLeafChunk, total - c0);
        const int cnp = (cn + 2 * L - 1) / (2 * L) * (2 * L);  // zero charges pad
        __syncthreads();
        for (int t = cn + threadIdx.x; t < cnp; t += kLeafThreads) {
          ps[t] = T4{T(0), T(0), T(0), T(0)};
          if constexpr (kSplit) pl[t] = float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int v = 1; v < NV; ++v) pq[v - 1][t] = T(0);
        }
        for (int t = threadIdx.x; t < cn; t += kLeafThreads) {
          const int g = c0 + t;
          int lo = 0, hi = nnb - 1;  // largest k with nb_pref[k] <= g
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (nb_pref[mid] <= g) lo = mid; else hi = mid - 1;
          }
          const int64_t si = (int64_t)nb_first[lo] + (g - nb_pref[lo]);
          const T q0 = vb < nvec ? (T)qs[(int64_t)vb * n_src + si] : T(0);
          const double ox = sxyz[3 * si] - cx, oy = sxyz[3 * si + 1] - cy, oz = sxyz[3 * si + 2] - cz;
          ps[t] = T4{(T)ox, (T)oy, (T)oz, q0};
          if constexpr (kSplit)
            pl[t] = float4{(float)(ox - (double)(T)ox), (float)(oy - (double)(T)oy),
                           (float)(oz - (double)(T)oz), 0.f};
#pragma unroll
          for (int v = 1; v < NV; ++v)
            pq[v - 1][t] = vb + v < nvec ? (T)qs[(int64_t)(vb + v) * n_src + si] : T(0);
        }
        __syncthreads();
        auto p2p = [&](int s) {
          const T4 src = ps[s];
          const T dx0 = xt0 - src.x, dy0 = yt0 - src.y, dz0 = zt0 - src.z;
          const T dx1 = xt1 - src.x, dy1 = yt1 - src.y, dz1 = zt1 - src.z;
          const T q0 = dx0 * dx0 + dy0 * dy0 + dz0 * dz0, q1 = dx1 * dx1 + dy1 * dy1 + dz1 * dz1;
          T r0 = inv_r(q0), r1 = inv_r(q1);
          if constexpr (kSplit) {
            if (q0 < tau2 || q1 < tau2) {  // rare: a pair closer than w / 16
              const float4 sl = pl[s];
              const float fx0 = dx0 + (xl0 - sl.x), fy0 = dy0 + (yl0 - sl.y), fz0 = dz0 + (zl0 - sl.z);
              const float fx1 = dx1 + (xl1 - sl.x), fy1 = dy1 + (yl1 - sl.y), fz1 = dz1 + (zl1 - sl.z);
              if (q0 < tau2) r0 = inv_r(fx0 * fx0 + fy0 * fy0 + fz0 * fz0);
              if (q1 < tau2) r1 = inv_r(fx1 * fx1 + fy1 * fy1 + fz1 * fz1);
            }
          }
          ap0[0] += r0 * src.w;
          ap1[0] += r1 * src.w;
#pragma unroll
          for (int v = 1; v < NV; ++v) {
            const T qv = pq[v - 1][s];
            ap0[v] += r0 * qv;
            ap1[v] += r1 * qv;
          }
        };
        for (int s0 = 0; s0 < cnp; s0 += 2 * L) {
          p2p(s0 + sub);
          p2p(s0 + L + sub);
        }
      }
      for (int off = 1; off < L; off <<= 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          al0[v] += __shfl_xor(al0[v], off);
          al1[v] += __shfl_xor(al1[v], off);
          ap0[v] += __shfl_xor(ap0[v], off);
          ap1[v] += __shfl_xor(ap1[v], off);
        }
      }
      if (sub == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (vb + v >= nvec) continue;
          if (MODE == 1) {
            // sorted target order: coalesced; the far-field pass scatters
            TQ* nr = static_cast<TQ*>(a.near) + (int64_t)(vb + v) * a.ldnear + t0;
            if (act0) nr[ti0] = (TQ)ap0[v];
            if (act1) nr[ti1] = (TQ)ap1[v];
          } else {
            TQ* o0 = act0 ? &phi[(int64_t)(vb + v) * ldphi + tperm[t0 + ti0]] : nullptr;
            TQ* o1 = act1 ? &phi[(int64_t)(vb + v) * ldphi + tperm[t0 + ti1]] : nullptr;
            const TQ* nr = MODE == 2 ? static_cast<const TQ*>(a.near) + (int64_t)(vb + v) * a.ldnear + t0
                                     : nullptr;
            const double n0 = MODE == 2 ? (o0 ? (double)nr[ti0] : 0.0) : (double)ap0[v];
            const double n1 = MODE == 2 ? (o1 ? (double)nr[ti1] : 0.0) : (double)ap1[v];
            if (o0) *o0 = (TQ)(kInv4Pi * (al0[v] + n0));
            if (o1) *o1 = (TQ)(kInv4Pi * (al1[v] + n1));
          }
        }
      }
    }
  }
}

template <typename T, typename TQ, int NV, int MODE>
__global__ __launch_bounds__(kLeafThreads) void leaf_eval_kernel(LeafArgs a) {
  leaf_eval_body<T, TQ, NV, MODE>(a, blockIdx.x);
}

template <typename T, typename TQ, int NV, int MODE>
__global__ __launch_bounds__(kLeafThreads) void leaf_eval_group_kernel(const LeafArgs* __restrict__ jobs,
                                                                      const int64_t* __restrict__ pre,
                                                                      int nj) {
  int64_t b;
  const LeafArgs a = jobs[group_job(pre, nj, b)];
  leaf_eval_body<T, TQ, NV, MODE>(a, b);
}

// Instance of the leaf kernel: (precision, mode, vector block).
int leaf_instance(bool fp64, int mode, int nvec) {
  const int nv = nvec == 1 ? 0 : nvec == 2 ? 1 : nvec <= 4 ? 2 : 3;
  return (fp64 ? 12 : 0) + mode * 4 + nv;
}

template <typename T, int NV, int MODE>
void leaf_go(const LeafArgs* one, const LeafArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
             hipStream_t s) {
  if (!jobs)
    leaf_eval_kernel<T, T, NV, MODE><<<(unsigned)blocks, kLeafThreads, 0, s>>>(*one);
  else
    leaf_eval_group_kernel<T, T, NV, MODE><<<(unsigned)blocks, kLeafThreads, 0, s>>>(jobs, pre, nj);
}

template <typename T, int MODE>
void leaf_go_nv(int nv, const LeafArgs* one, const LeafArgs* jobs, const int64_t* pre, int nj,
                int64_t blocks, hipStream_t s) {
  if (nv == 0) leaf_go<T, 1, MODE>(one, jobs, pre, nj, blocks, s);
  else if (nv == 1) leaf_go<T, 2, MODE>(one, jobs, pre, nj, blocks, s);
  else if (nv == 2) leaf_go<T, 4, MODE>(one, jobs, pre, nj, blocks, s);
  else leaf_go<T, 8, MODE>(one, jobs, pre, nj, blocks, s);
}

template <typename T>
void leaf_go_mode(int mode, int nv, const LeafArgs* one, const LeafArgs* jobs, const int64_t* pre,
                  int nj, int64_t blocks, hipStream_t s) {
  if (mode == 0) leaf_go_nv<T, 0>(nv, one, jobs, pre, nj, blocks, s);
  else if (mode == 1) leaf_go_nv<T, 1>(nv, one, jobs, pre, nj, blocks, s);
  else leaf_go_nv<T, 2>(nv, one, jobs, pre, nj, blocks, s);
}

hipError_t leaf_dispatch(int inst, const LeafArgs* one, const LeafArgs* jobs, const int64_t* pre, int nj,
                         int64_t blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (inst < 0 || inst >= 24 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int mode = (inst % 12) / 4, nv = inst % 4;
  if (inst >= 12)
    leaf_go_mode<double>(mode, nv, one, jobs, pre, nj, blocks, s);
  else
    leaf_go_mode<float>(mode, nv, one, jobs, pre, nj, blocks, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(const void* q, int64_t ldq, const int64_t* perm, int64_t n, int nvec,
                         bool fp64, void* qs, hipStream_t stream) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nvec);
  if (fp64)
    gather_kernel<double><<<grid, 256, 0, stream>>>((const double*)q, ldq, perm, n, (double*)qs);
  else
    gather_kernel<float><<<grid, 256, 0, stream>>>((const float*)q, ldq, perm, n, (float*)qs);
  return hipGetLastError();
}

hipError_t launch_p2m(const double* src_xyz, const void* qs, bool q_fp64, int64_t n_src,
                      const int32_t* start, const int32_t* end, const double* centers, int64_t n_leaf,
                      const double* surf, double ar, int ns, int nvec, double* phi,
                      hipStream_t stream) {
  P2MArgs a;
  int inst;
  int64_t blocks;
  plan_p2m(src_xyz, qs, q_fp64, n_src, start, end, centers, n_leaf, surf, ar, ns, nvec, phi, a, inst,
           blocks);
  return p2m_dispatch(inst, &a, nullptr, nullptr, 0, blocks, stream);
}

void plan_p2m(const double* src_xyz, const void* qs, bool q_fp64, int64_t n_src, const int32_t* start,
              const int32_t* end, const double* centers, int64_t n_leaf, const double* surf, double ar,
              int ns, int nvec, double* phi, P2MArgs& a, int& inst, int64_t& blocks) {
  a = P2MArgs{src_xyz, qs, n_src, start, end, centers, surf, ar, ns, nvec, phi, n_leaf};
  inst = p2m_instance(q_fp64, ns, nvec);
  blocks = n_leaf;
}

hipError_t launch_p2m_group(int inst, const P2MArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
                            hipStream_t stream) {
  return p2m_dispatch(inst, nullptr, jobs, pre, nj, blocks, stream);
}

void plan_leaf_eval(const double* tgt_xyz, const double* src_xyz, double leaf_w, const void* qs,
                    bool fp64, int64_t n_src, const int32_t* tstart, const int32_t* tend,
                    const int32_t* sstart, const int32_t* send, const int64_t* near_offs,
                    const int32_t* near_src, const double* centers, int64_t n_leaf,
                    const double* surf, double ar, int ns, const double* local,
                    const int64_t* tgt_perm, void* phi, int64_t ldphi, void* near, int64_t ldnear,
                    int nvec, int mode, LeafArgs& a, int& inst, int64_t& blocks) {
  const double tau2 = (leaf_w / 16) * (leaf_w / 16);  // FP32: pairs refined below w / 16
  a = LeafArgs{tgt_xyz, src_xyz, qs, n_src, tstart, tend, sstart, send, near_offs, near_src, centers,
               surf, ar, ns, local, tgt_perm, phi, ldphi, nvec, n_leaf, tau2, near, ldnear};
  inst = (mode < 0 || mode > 2) ? -1 : leaf_instance(fp64, mode, nvec);
  blocks = 8 * ((n_leaf + 7) / 8);
}

hipError_t launch_leaf_eval(const double* tgt_xyz, const double* src_xyz, double leaf_w,
                            const void* qs, bool fp64, int64_t n_src, const int32_t* tstart,
                            const int32_t* tend, const int32_t* sstart, const int32_t* send,
                            const int64_t* near_offs, const int32_t* near_src,
                            const double* centers, int64_t n_leaf, const double* surf, double ar,
                            int ns, const double* local, const int64_t* tgt_perm, void* phi,
                            int64_t ldphi, void* near, int64_t ldnear, int nvec, int mode,
                            hipStream_t stream) {
  if (n_leaf == 0) return hipSuccess;
  if (mode != 0 && !near) return hipErrorInvalidValue;
  LeafArgs a;
  int inst;
  int64_t blocks;
  plan_leaf_eval(tgt_xyz, src_xyz, leaf_w, qs, fp64, n_src, tstart, tend, sstart, send, near_offs,
                 near_src, centers, n_leaf, surf, ar, ns, local, tgt_perm, phi, ldphi, near, ldnear,
                 nvec, mode, a, inst, blocks);
  return leaf_dispatch(inst, &a, nullptr, nullptr, 0, blocks, stream);
}

hipError_t launch_leaf_eval_group(int inst, const LeafArgs* jobs, const int64_t* pre, int nj,
                                  int64_t blocks, hipStream_t stream) {
  return leaf_dispatch(inst, nullptr, jobs, pre, nj, blocks, stream);
}

hipError_t launch_gather_group(bool fp64, const GatherArgs* jobs, const int64_t* pre, int nj,
                               int64_t blocks, hipStream_t stream) {
  if (blocks == 0) return hipSuccess;
  if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (fp64)
    gather_group_kernel<double><<<(unsigned)blocks, 256, 0, stream>>>(jobs, pre, nj);
  else
    gather_group_kernel<float><<<(unsigned)blocks, 256, 0, stream>>>(jobs, pre, nj);
  return hipGetLastError();
}

}  // namespace kifmm
