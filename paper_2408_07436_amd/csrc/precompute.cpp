// FP64 host precomputation of the kiFMM operators for a box of unit width.
//
// Surfaces and pseudo-inverses follow Section 2.1.1 of arXiv 2408.07436,
// M2M/L2L the translation operators of Section 2.2, FFT kernel spectra the
// convolution grid of Appendix A.1 (real-kernel halving of Appendix A.2),
// and the SVD compression with directional recompression Section 3.1.
//
// The Laplace kernel is homogeneous of degree -1, so every operator of a box
// of width w equals the unit-box operator divided by w (pseudo-inverses are
// multiplied by w); the device code applies that scale per level.
#include <cmath>
#include <algorithm>
#include <atomic>
#include <complex>
#include <thread>

#include "internal.h"

namespace kifmm {

namespace {
// Runs f(i) for i in [0, n) on up to 16 host threads (independent items).
template <typename F>
void parallel_for(int n, F f) {
  const int nt = std::max(1, std::min({n, 16, (int)std::thread::hardware_concurrency()}));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i = next++; i < n; i = next++) f(i);
  };
  std::vector<std::thread> pool;
  for (int k = 1; k < nt; ++k) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
}
}  // namespace

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

double lap(const double* x, const double* y) {
  const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
  const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  return r == 0.0 ? 0.0 : kInv4Pi / r;
}

// points c + alpha * r * s_i of a surface given by its unit offsets
std::vector<double> place_on(const std::vector<double>& surf, double alpha, double r, const double c[3]) {
  std::vector<double> pts(surf.size());
  const double ar = alpha * r;
  for (size_t i = 0; i < surf.size() / 3; ++i)
    for (int k = 0; k < 3; ++k) pts[3 * i + k] = c[k] + ar * surf[3 * i + k];
  return pts;
}
// equivalent surface (order p) and check surface (order pc)
std::vector<double> place(const Operators& op, double alpha, double r, const double c[3]) {
  return place_on(op.surf, alpha, r, c);
}
std::vector<double> place_c(const Operators& op, double alpha, double r, const double c[3]) {
  return place_on(op.surf_c, alpha, r, c);
}

// boundary points of the q x q x q lattice, i_x slowest: unit offsets
// -1 + 2 i / (q - 1) and (optionally) the integer positions
void lattice_surface(int q, std::vector<double>& surf, std::vector<int32_t>* lattice) {
  surf.clear();
  if (lattice) lattice->clear();
  for (int ix = 0; ix < q; ++ix)
    for (int iy = 0; iy < q; ++iy)
      for (int iz = 0; iz < q; ++iz) {
        const bool bnd = ix == 0 || iy == 0 || iz == 0 || ix == q - 1 || iy == q - 1 || iz == q - 1;
        if (!bnd) continue;
        const int id[3] = {ix, iy, iz};
        for (int k = 0; k < 3; ++k) {
          if (lattice) lattice->push_back(id[k]);
          surf.push_back(-1.0 + 2.0 * id[k] / (q - 1));
        }
      }
}

void kernel_block(const std::vector<double>& x, const std::vector<double>& y, int nx, int ny,
                  double* out, int ld) {
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < ny; ++j) out[(size_t)i * ld + j] = lap(&x[3 * i], &y[3 * j]);
}

// two-factor pseudo-inverse (Section 2.1.1): keep sigma > max(m,n) eps sigma_0
kifmm_status pinv(const std::vector<double>& K, int m, int n, int& rank, std::vector<double>& V,
                  std::vector<double>& Ut) {
  std::vector<double> U, s, W;
  if (!svd(K.data(), m, n, U, s, W)) return fail(KIFMM_ENUMERIC, "Jacobi SVD did not converge");
  const int r0 = std::min(m, n);
  const double tol = std::max(m, n) * 2.220446049250313e-16 * s[0];
  rank = 0;
  while (rank < r0 && s[rank] > tol) ++rank;
  V.assign((size_t)n * rank, 0.0);
  Ut.assign((size_t)rank * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < rank; ++j) V[(size_t)i * rank + j] = W[(size_t)i * r0 + j];
  for (int j = 0; j < rank; ++j)
    for (int i = 0; i < m; ++i) Ut[(size_t)j * m + i] = U[(size_t)i * r0 + j] / s[j];
  return KIFMM_OK;
}

// r2c DFT of a real (n x n x n) grid, output [kx][ky][kz], kz in [0, n/2]
void rdft3(const std::vector<double>& g, int n, std::vector<std::complex<double>>& out) {
  const int h = n / 2 + 1;
  std::vector<std::complex<double>> w(n);
  for (int m = 0; m < n; ++m) w[m] = std::polar(1.0, -2.0 * M_PI * m / n);
  std::vector<std::complex<double>> a((size_t)n * n * h), b((size_t)n * n * h);
  for (int x = 0; x < n; ++x)
    for (int y = 0; y < n; ++y)
      for (int kz = 0; kz < h; ++kz) {
        std::complex<double> acc = 0;
        for (int z = 0; z < n; ++z) acc += g[((size_t)x * n + y) * n + z] * w[(kz * z) % n];
        a[((size_t)x * n + y) * h + kz] = acc;
      }
  for (int x = 0; x < n; ++x)
    for (int ky = 0; ky < n; ++ky)
      for (int kz = 0; kz < h; ++kz) {
        std::complex<double> acc = 0;
        for (int y = 0; y < n; ++y) acc += a[((size_t)x * n + y) * h + kz] * w[(ky * y) % n];
        b[((size_t)x * n + ky) * h + kz] = acc;
      }
  out.assign((size_t)n * n * h, 0);
  for (int kx = 0; kx < n; ++kx)
    for (int ky = 0; ky < n; ++ky)
      for (int kz = 0; kz < h; ++kz) {
        std::complex<double> acc = 0;
        for (int x = 0; x < n; ++x) acc += b[((size_t)x * n + ky) * h + kz] * w[(kx * x) % n];
        out[((size_t)kx * n + ky) * h + kz] = acc;
      }
}

}  // namespace

kifmm_status precompute_operators(Operators& op, const kifmm_config& cfg, const SvdOptions& svd_opt) {
  op = Operators();
  const int p = cfg.order;
  const int pc = cfg.check_order > 0 ? cfg.check_order : p;
  if (pc < p) return fail(KIFMM_EINVAL, "check order below the expansion order");
  if (pc != p && cfg.m2l != KIFMM_M2L_BLAS)
    return fail(KIFMM_EUNSUPPORTED, "a check order above the expansion order needs BLAS-M2L");
  op.p = p;
  op.pc = pc;
  op.ai = cfg.alpha_inner > 0 ? cfg.alpha_inner : 1.05;
  op.ao = cfg.alpha_outer > 0 ? cfg.alpha_outer : 2.95;
  lattice_surface(p, op.surf, &op.lattice);
  op.ns = (int)op.lattice.size() / 3;
  if (pc == p)
    op.surf_c = op.surf;
  else
    lattice_surface(pc, op.surf_c, nullptr);
  op.nc = (int)op.surf_c.size() / 3;
  // convolution grid of 2p - 1 points per axis: the offsets of check and
  // equivalent lattice points span 2p - 1 values, so the circular
  // convolution does not wrap (the paper pads to 2p)
  op.n = 2 * p - 1;
  op.F = op.n * op.n * (op.n / 2 + 1);
  const int ns = op.ns, nc = op.nc;
  const double zero[3] = {0, 0, 0};

  // pseudo-inverses of the unit box: up K(UC, UE), down K(DC, DE) (nc x ns)
  {
    std::vector<double> K((size_t)nc * ns);
    kernel_block(place_c(op, op.ao, 0.5, zero), place(op, op.ai, 0.5, zero), nc, ns, K.data(), ns);
    kifmm_status st = pinv(K, nc, ns, op.r_up, op.up_V, op.up_Ut);
    if (st != KIFMM_OK) return st;
    kernel_block(place_c(op, op.ai, 0.5, zero), place(op, op.ao, 0.5, zero), nc, ns, K.data(), ns);
    st = pinv(K, nc, ns, op.r_down, op.down_V, op.down_Ut);
    if (st != KIFMM_OK) return st;
  }
  // M2M [K_0 .. K_7] (nc x 8 ns) and L2L [L_0; ..; L_7] (8 nc x ns) for a
  // parent of width 1
  op.m2m.assign((size_t)nc * 8 * ns, 0.0);
  op.l2l.assign((size_t)8 * nc * ns, 0.0);
  {
    const auto uc = place_c(op, op.ao, 0.5, zero);
    const auto de = place(op, op.ao, 0.5, zero);
    for (int o = 0; o < 8; ++o) {
      const double c[3] = {(((o >> 0) & 1) - 0.5) * 0.5, (((o >> 1) & 1) - 0.5) * 0.5,
                           (((o >> 2) & 1) - 0.5) * 0.5};
      kernel_block(uc, place(op, op.ai, 0.25, c), nc, ns, &op.m2m[(size_t)o * ns], 8 * ns);
      kernel_block(place_c(op, op.ai, 0.25, c), de, nc, ns, &op.l2l[(size_t)o * nc * ns], ns);
    }
  }

  // composite operators (products accumulated in extended precision)
  {
    auto matmul = [](const double* A, const double* B, int m, int k, int n, int lda, int ldb,
                     double* C, int ldc) {
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
          long double acc = 0.0L;
          for (int t = 0; t < k; ++t) acc += (long double)A[(size_t)i * lda + t] * B[(size_t)t * ldb + j];
          C[(size_t)i * ldc + j] = (double)acc;
        }
    };
    op.up_P.assign((size_t)ns * nc, 0.0);
    op.down_P.assign((size_t)ns * nc, 0.0);
    matmul(op.up_V.data(), op.up_Ut.data(), ns, op.r_up, nc, op.r_up, nc, op.up_P.data(), nc);
    matmul(op.down_V.data(), op.down_Ut.data(), ns, op.r_down, nc, op.r_down, nc, op.down_P.data(), nc);
    op.m2m_c.assign((size_t)ns * 8 * ns, 0.0);
    matmul(op.up_P.data(), op.m2m.data(), ns, nc, 8 * ns, nc, 8 * ns, op.m2m_c.data(), 8 * ns);
    op.l2l_c.assign((size_t)8 * ns * ns, 0.0);
    for (int o = 0; o < 8; ++o)
      matmul(op.down_P.data(), &op.l2l[(size_t)o * nc * ns], ns, nc, ns, nc, ns,
             &op.l2l_c[(size_t)o * ns * ns], ns);
  }

  if (cfg.m2l == KIFMM_M2L_FFT) {
    // kernel sequences G[m] = K(c_tau - c_sigma + h m) on the (2p-1)^3 grid
    const int n = op.n;
    const double h = 2.0 * op.ai * 0.5 / (p - 1);
    op.spectra.assign((size_t)kNumTransfer * op.F * 2, 0.0);
    std::vector<double> g((size_t)n * n * n);
    std::vector<std::complex<double>> spec;
    for (int it = 0; it < kNumTransfer; ++it) {
      int t[3];
      transfer_vector(it, t);
      std::fill(g.begin(), g.end(), 0.0);
      for (int mx = -(p - 1); mx <= p - 1; ++mx)
        for (int my = -(p - 1); my <= p - 1; ++my)
          for (int mz = -(p - 1); mz <= p - 1; ++mz) {
            const double d[3] = {-t[0] + h * mx, -t[1] + h * my, -t[2] + h * mz};
            const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            g[(((size_t)((mx + n) % n) * n) + (my + n) % n) * n + (mz + n) % n] = kInv4Pi / r;
          }
      rdft3(g, n, spec);
      for (int f = 0; f < op.F; ++f) {
        op.spectra[((size_t)it * op.F + f) * 2] = spec[f].real();
        op.spectra[((size_t)it * op.F + f) * 2 + 1] = spec[f].imag();
      }
    }
  } else {
    // M2L matrices K_t of the unit box (check surface around 0, equivalent
    // surface around t), both on the inner surface; nc x ns
    const auto dc = place_c(op, op.ai, 0.5, zero);
    std::vector<std::vector<double>> Kt(kNumTransfer, std::vector<double>((size_t)nc * ns));
    parallel_for(kNumTransfer, [&](int it) {
      int t[3];
      transfer_vector(it, t);
      const double c[3] = {(double)t[0], (double)t[1], (double)t[2]};
      kernel_block(dc, place(op, op.ai, 0.5, c), nc, ns, Kt[it].data(), ns);
    });
    op.Ubar.assign(kNumTransfer, {});
    op.Vbarp.assign(kNumTransfer, {});
    op.kt.assign(kNumTransfer, 0);
    if (cfg.m2l == KIFMM_M2L_DENSE) {
      op.k = ns;
      op.U.assign((size_t)ns * ns, 0.0);
      for (int i = 0; i < ns; ++i) op.U[(size_t)i * ns + i] = 1.0;
      op.S = op.U;
      for (int it = 0; it < kNumTransfer; ++it) {
        op.kt[it] = ns;
        op.Vbarp[it] = Kt[it];  // applied directly as C_t = K_t
      }
      op.recompressed = false;
    } else {
      // K_fat = [K_1 .. K_T] (nc x T ns): its left vectors give U.  With
      // nc = ns, K_t^T = K_{-t} makes K_thin's right vectors equal K_fat's
      // left vectors, so S = U (Section 3.1, symmetric kernels); otherwise S
      // comes from the left vectors of K_thin^T = [K_1^T .. K_T^T] (ns x T nc).
      auto left = [&](const std::vector<double>& A, int m, int n, std::vector<double>& Uo,
                      std::vector<double>& so) -> kifmm_status {
        if (svd_opt.mode == KIFMM_SVD_RANDOMIZED) return rsvd_left_device(A.data(), m, n, svd_opt, Uo, so);
        if (!svd_left_wide(A.data(), m, n, Uo, so)) return fail(KIFMM_ENUMERIC, "SVD of K_fat / K_thin did not converge");
        return KIFMM_OK;
      };
      std::vector<double> Kfat((size_t)nc * kNumTransfer * ns);
      for (int i = 0; i < nc; ++i)
        for (int it = 0; it < kNumTransfer; ++it)
          std::copy(&Kt[it][(size_t)i * ns], &Kt[it][(size_t)i * ns] + ns,
                    &Kfat[((size_t)i * kNumTransfer + it) * ns]);
      std::vector<double> Uf, sf;
      kifmm_status st = left(Kfat, nc, kNumTransfer * ns, Uf, sf);
      if (st != KIFMM_OK) return st;
      const int r0 = (int)sf.size();
      int k = 0;
      if (cfg.svd_rel_tol > 0) {
        while (k < r0 && sf[k] > cfg.svd_rel_tol * sf[0]) ++k;
      } else {
        while (k < r0 && sf[k] > 0.0) ++k;
      }
      std::vector<double> Sf;
      int rs = r0;
      if (nc == ns) {
        Sf = Uf;
      } else {
        std::vector<double> KthinT((size_t)ns * kNumTransfer * nc), ss;
        for (int it = 0; it < kNumTransfer; ++it)
          for (int i = 0; i < nc; ++i)
            for (int j = 0; j < ns; ++j) KthinT[((size_t)j * kNumTransfer + it) * nc + i] = Kt[it][(size_t)i * ns + j];
        st = left(KthinT, ns, kNumTransfer * nc, Sf, ss);
        if (st != KIFMM_OK) return st;
        rs = (int)ss.size();
        k = std::min(k, rs);
      }
      op.k = k;
      op.U.assign((size_t)nc * k, 0.0);
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < k; ++j) op.U[(size_t)i * k + j] = Uf[(size_t)i * r0 + j];
      op.S.assign((size_t)ns * k, 0.0);
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < k; ++j) op.S[(size_t)i * k + j] = Sf[(size_t)i * rs + j];
      op.recompressed = cfg.svd_rel_tol_dir >= 0;
      // the transfer vectors are independent: one host thread each at a time
      std::atomic<bool> svd_failed{false};
      parallel_for(kNumTransfer, [&](int it) {
        std::vector<double> tmp((size_t)nc * k), C((size_t)k * k);
        // C_t = U^T K_t S
        for (int i = 0; i < nc; ++i)
          for (int j = 0; j < k; ++j) {
            double acc = 0;
            for (int l = 0; l < ns; ++l) acc += Kt[it][(size_t)i * ns + l] * op.S[(size_t)l * k + j];
            tmp[(size_t)i * k + j] = acc;
          }
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < k; ++j) {
            double acc = 0;
            for (int l = 0; l < nc; ++l) acc += op.U[(size_t)l * k + i] * tmp[(size_t)l * k + j];
            C[(size_t)i * k + j] = acc;
          }
        if (!op.recompressed) {
          op.kt[it] = k;
          op.Vbarp[it] = C;  // applied directly
          return;
        }
        std::vector<double> cu, cs, cv;
        if (!svd(C.data(), k, k, cu, cs, cv)) {
          svd_failed = true;
          return;
        }
        int r = 0;
        while (r < k && cs[r] > cfg.svd_rel_tol_dir * cs[0]) ++r;
        if (r == 0) r = 1;
        op.kt[it] = r;
        op.Ubar[it].assign((size_t)k * r, 0.0);
        op.Vbarp[it].assign((size_t)k * r, 0.0);
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < r; ++j) {
            op.Ubar[it][(size_t)i * r + j] = cu[(size_t)i * k + j];
            op.Vbarp[it][(size_t)i * r + j] = cv[(size_t)i * k + j] * cs[j];
          }
      });
      if (svd_failed) return fail(KIFMM_ENUMERIC, "SVD of C_t did not converge");
    }
  }
  op.ready = true;
  return KIFMM_OK;
}

}  // namespace kifmm
