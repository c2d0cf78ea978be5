// Point kernels of the kiFMM on gfx950: charge gather into Morton order,
// P2M check potentials (Section 2.1.1) and the fused leaf evaluation
// L2P + P2P (Section 2, downward pass).  Laplace kernel 1 / (4 pi r), zero
// at r = 0.
#include "kernels.h"

namespace kifmm {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;

__device__ inline double inv_r(double r2) { return r2 > 0.0 ? rsqrt(r2) : 0.0; }
__device__ inline float inv_r(float r2) { return r2 > 0.0f ? rsqrtf(r2) : 0.0f; }

template <typename TQ>
__global__ void gather_kernel(const TQ* __restrict__ q, int64_t ldq, const int64_t* __restrict__ perm,
                              int64_t n, TQ* __restrict__ qs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (i < n) qs[v * n + i] = q[v * ldq + perm[i]];
}

constexpr int kP2MThreads = 256;
constexpr int kP2MChunk = 64;
constexpr int kP2MVec = 8;

// One workgroup per leaf; a thread owns one upward-check point and
// accumulates up to kP2MVec charge vectors at a time.
template <typename TQ>
__global__ __launch_bounds__(kP2MThreads) void p2m_kernel(
    const double* __restrict__ xyz, const TQ* __restrict__ qs, int64_t n_src,
    const int32_t* __restrict__ start, const int32_t* __restrict__ end,
    const double* __restrict__ centers, const double* __restrict__ surf, double ar, int ns, int nvec,
    double* __restrict__ phi) {
  __shared__ double sx[kP2MChunk], sy[kP2MChunk], sz[kP2MChunk];
  __shared__ double sq[kP2MVec][kP2MChunk];
  const int64_t leaf = blockIdx.x;
  const int s0 = start[leaf], s1 = end[leaf];
  const double cx = centers[3 * leaf], cy = centers[3 * leaf + 1], cz = centers[3 * leaf + 2];
  for (int i0 = 0; i0 < ns; i0 += kP2MThreads) {
    const int i = i0 + (int)threadIdx.x;
    const bool act = i < ns;
    double px = 0, py = 0, pz = 0;
    if (act) {
      px = cx + ar * surf[3 * i];
      py = cy + ar * surf[3 * i + 1];
      pz = cz + ar * surf[3 * i + 2];
    }
    for (int vb = 0; vb < nvec; vb += kP2MVec) {
      double acc[kP2MVec];
#pragma unroll
      for (int v = 0; v < kP2MVec; ++v) acc[v] = 0.0;
      for (int c0 = s0; c0 < s1; c0 += kP2MChunk) {
        const int cn = min(kP2MChunk, s1 - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kP2MThreads) {
          sx[t] = xyz[3 * (int64_t)(c0 + t)];
          sy[t] = xyz[3 * (int64_t)(c0 + t) + 1];
          sz[t] = xyz[3 * (int64_t)(c0 + t) + 2];
        }
        for (int t = threadIdx.x; t < kP2MVec * kP2MChunk; t += kP2MThreads) {
          const int v = t / kP2MChunk, s = t % kP2MChunk;
          sq[v][s] = (s < cn && vb + v < nvec) ? (double)qs[(int64_t)(vb + v) * n_src + c0 + s] : 0.0;
        }
        __syncthreads();
        if (act) {
          for (int s = 0; s < cn; ++s) {
            const double dx = px - sx[s], dy = py - sy[s], dz = pz - sz[s];
            const double ir = inv_r(dx * dx + dy * dy + dz * dz);
#pragma unroll
            for (int v = 0; v < kP2MVec; ++v) acc[v] += ir * sq[v][s];
          }
        }
      }
      if (act) {
#pragma unroll
        for (int v = 0; v < kP2MVec; ++v)
          if (vb + v < nvec) phi[((int64_t)leaf * nvec + vb + v) * ns + i] = kInv4Pi * acc[v];
      }
    }
  }
}

constexpr int kLeafThreads = 128;
constexpr int kLeafVec = 4;
constexpr int kLeafChunk = 256;  // near-field sources staged per pass
constexpr int kL2PChunk = 160;   // downward-equivalent points staged per pass

// One workgroup per target leaf.  The near-field sources (up to 27 leaves,
// each a contiguous run in Morton order) are staged through LDS in chunks;
// a thread finds the run of a staged source by binary search over the run
// offsets.  1, 2 or 4 lanes share a target (by leaf occupancy), split the
// staged sources and reduce with cross-lane shuffles.  L2P runs in FP64 from
// the leaf's downward-equivalent densities; P2P runs in T.
template <typename T, typename TQ>
__global__ __launch_bounds__(kLeafThreads) void leaf_eval_kernel(
    const double* __restrict__ txyz, const T* __restrict__ sxyz, const TQ* __restrict__ qs,
    int64_t n_src, const int32_t* __restrict__ tstart, const int32_t* __restrict__ tend,
    const int32_t* __restrict__ sstart, const int32_t* __restrict__ send,
    const int64_t* __restrict__ noffs, const int32_t* __restrict__ nsrc,
    const double* __restrict__ centers, const double* __restrict__ surf, double ar, int ns,
    const double* __restrict__ local, const int64_t* __restrict__ tperm, TQ* __restrict__ phi,
    int64_t ldphi, int nvec) {
  __shared__ double lx[kL2PChunk], ly[kL2PChunk], lz[kL2PChunk];
  __shared__ double lq[kLeafVec][kL2PChunk];
  __shared__ T px[kLeafChunk], py[kLeafChunk], pz[kLeafChunk];
  __shared__ T pq[kLeafVec][kLeafChunk];
  __shared__ int32_t nb_first[27];
  __shared__ int32_t nb_pref[28];
  __shared__ int32_t n_nb;

  const int64_t leaf = blockIdx.x;
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
  const int L = nt <= 32 ? 4 : (nt <= 64 ? 2 : 1);
  const int slots = kLeafThreads / L;
  const int tt = threadIdx.x / L, sub = threadIdx.x % L;
  const double cx = centers[3 * leaf], cy = centers[3 * leaf + 1], cz = centers[3 * leaf + 2];

  for (int vb = 0; vb < nvec; vb += kLeafVec) {
    for (int tb = 0; tb < nt; tb += slots) {
      const int ti = tb + tt;
      const bool act = ti < nt;
      double x = 0, y = 0, z = 0;
      if (act) {
        x = txyz[3 * (int64_t)(t0 + ti)];
        y = txyz[3 * (int64_t)(t0 + ti) + 1];
        z = txyz[3 * (int64_t)(t0 + ti) + 2];
      }
      double accl[kLeafVec];
      T accp[kLeafVec];
#pragma unroll
      for (int v = 0; v < kLeafVec; ++v) {
        accl[v] = 0.0;
        accp[v] = T(0);
      }
      // L2P: the leaf's downward-equivalent surface as sources (FP64)
      for (int c0 = 0; c0 < ns; c0 += kL2PChunk) {
        const int cn = min(kL2PChunk, ns - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kLeafThreads) {
          lx[t] = cx + ar * surf[3 * (c0 + t)];
          ly[t] = cy + ar * surf[3 * (c0 + t) + 1];
          lz[t] = cz + ar * surf[3 * (c0 + t) + 2];
#pragma unroll
          for (int v = 0; v < kLeafVec; ++v)
            lq[v][t] = vb + v < nvec ? local[((int64_t)leaf * nvec + vb + v) * ns + c0 + t] : 0.0;
        }
        __syncthreads();
        if (act) {
          for (int s = sub; s < cn; s += L) {
            const double dx = x - lx[s], dy = y - ly[s], dz = z - lz[s];
            const double ir = inv_r(dx * dx + dy * dy + dz * dz);
#pragma unroll
            for (int v = 0; v < kLeafVec; ++v) accl[v] += ir * lq[v][s];
          }
        }
      }
      // P2P over the near field
      const T xt = (T)x, yt = (T)y, zt = (T)z;
      for (int c0 = 0; c0 < total; c0 += kLeafChunk) {
        const int cn = min(kLeafChunk, total - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += kLeafThreads) {
          const int g = c0 + t;
          int lo = 0, hi = nnb - 1;  // largest k with nb_pref[k] <= g
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (nb_pref[mid] <= g) lo = mid; else hi = mid - 1;
          }
          const int64_t si = (int64_t)nb_first[lo] + (g - nb_pref[lo]);
          px[t] = sxyz[3 * si];
          py[t] = sxyz[3 * si + 1];
          pz[t] = sxyz[3 * si + 2];
#pragma unroll
          for (int v = 0; v < kLeafVec; ++v)
            pq[v][t] = vb + v < nvec ? (T)qs[(int64_t)(vb + v) * n_src + si] : T(0);
        }
        __syncthreads();
        if (act) {
          for (int s = sub; s < cn; s += L) {
            const T dx = xt - px[s], dy = yt - py[s], dz = zt - pz[s];
            const T ir = inv_r(dx * dx + dy * dy + dz * dz);
#pragma unroll
            for (int v = 0; v < kLeafVec; ++v) accp[v] += ir * pq[v][s];
          }
        }
      }
      for (int off = 1; off < L; off <<= 1) {
#pragma unroll
        for (int v = 0; v < kLeafVec; ++v) {
          accl[v] += __shfl_xor(accl[v], off);
          accp[v] += __shfl_xor(accp[v], off);
        }
      }
      if (act && sub == 0) {
        const int64_t dst = tperm[t0 + ti];
#pragma unroll
        for (int v = 0; v < kLeafVec; ++v)
          if (vb + v < nvec)
            phi[(int64_t)(vb + v) * ldphi + dst] = (TQ)(kInv4Pi * (accl[v] + (double)accp[v]));
      }
    }
  }
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
  if (n_leaf == 0) return hipSuccess;
  if (q_fp64)
    p2m_kernel<double><<<(unsigned)n_leaf, kP2MThreads, 0, stream>>>(
        src_xyz, (const double*)qs, n_src, start, end, centers, surf, ar, ns, nvec, phi);
  else
    p2m_kernel<float><<<(unsigned)n_leaf, kP2MThreads, 0, stream>>>(
        src_xyz, (const float*)qs, n_src, start, end, centers, surf, ar, ns, nvec, phi);
  return hipGetLastError();
}

hipError_t launch_leaf_eval(const double* tgt_xyz, const double* src_xyz, const float* src_xyz_f,
                            const void* qs, bool fp64, int64_t n_src, const int32_t* tstart,
                            const int32_t* tend, const int32_t* sstart, const int32_t* send,
                            const int64_t* near_offs, const int32_t* near_src,
                            const double* centers, int64_t n_leaf, const double* surf, double ar,
                            int ns, const double* local, const int64_t* tgt_perm, void* phi,
                            int64_t ldphi, int nvec, hipStream_t stream) {
  if (n_leaf == 0) return hipSuccess;
  if (fp64)
    leaf_eval_kernel<double, double><<<(unsigned)n_leaf, kLeafThreads, 0, stream>>>(
        tgt_xyz, src_xyz, (const double*)qs, n_src, tstart, tend, sstart, send, near_offs,
        near_src, centers, surf, ar, ns, local, tgt_perm, (double*)phi, ldphi, nvec);
  else
    leaf_eval_kernel<float, float><<<(unsigned)n_leaf, kLeafThreads, 0, stream>>>(
        tgt_xyz, src_xyz_f, (const float*)qs, n_src, tstart, tend, sstart, send, near_offs,
        near_src, centers, surf, ar, ns, local, tgt_perm, (float*)phi, ldphi, nvec);
  return hipGetLastError();
}

}  // namespace kifmm
