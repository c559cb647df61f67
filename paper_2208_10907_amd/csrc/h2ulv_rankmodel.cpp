// Learned rank prediction (internal): box features and the rank model's
// host-side management (initialisation, training loop).  The network's forward
// pass, gradient and Adam update are the kernels of h2ulv_learned.hip.
#include <cmath>
#include <cstring>

#include "h2ulv_factor.h"
#include "h2ulv_learned.h"

namespace h2ulv {

namespace {

// Eigenvalues of a symmetric 3 x 3 matrix by cyclic Jacobi rotations.
void sym3_eigenvalues(double a[3][3], double ev[3]) {
  const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int r = 0; r < 3; ++r) {
      const int p = P[r], q = Q[r];
      const double apq = a[p][q];
      if (std::fabs(apq) < 1e-300) continue;
      // rotation in the (p, q) plane that zeroes a[p][q]
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      const int o = 3 - p - q;
      const double aop = a[o][p], aoq = a[o][q];
      a[o][p] = a[p][o] = c * aop - s * aoq;
      a[o][q] = a[q][o] = s * aop + c * aoq;
    }
  }
  for (int i = 0; i < 3; ++i) ev[i] = a[i][i];
}

double host_gauss(uint64_t key, uint64_t i) {
  const uint64_t x1 = sm64_at(key, 2 * i), x2 = sm64_at(key, 2 * i + 1);
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
}

}  // namespace

void box_features(const h2ulv_factor& F, int lev, int i, int m, int ntargets, int64_t ncols,
                  double child_ratio, float* out) {
  const Tree& T = F.tree;
  const Lists& ls = F.lists;
  const int64_t s0 = T.start[lev][i], s1 = T.end[lev][i];
  const int64_t np = s1 - s0;
  double mu[3] = {0, 0, 0};
  for (int64_t a = s0; a < s1; ++a)
    for (int d = 0; d < 3; ++d) mu[d] += F.hpts[3 * T.perm[a] + d];
  for (int d = 0; d < 3; ++d) mu[d] /= (double)np;
  double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int64_t a = s0; a < s1; ++a) {
    double x[3];
    for (int d = 0; d < 3; ++d) x[d] = F.hpts[3 * T.perm[a] + d] - mu[d];
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e) C[d][e] += x[d] * x[e];
  }
  for (int d = 0; d < 3; ++d)
    for (int e = 0; e < 3; ++e) C[d][e] /= (double)np;
  double ev[3];
  sym3_eigenvalues(C, ev);
  std::sort(ev, ev + 3, [](double x, double y) { return x > y; });
  const double r = T.radius[lev][i], r0 = T.radius[0][0];
  const h2ulv_params& p = F.p;
  double f[16];
  f[0] = std::log2(1.0 + m) / 12.0;
  f[1] = std::log2(1.0 + (double)np) / 20.0;
  f[2] = (double)lev / (double)std::max(T.L, 1);
  f[3] = std::log2(1.0 + (double)(ls.near_ptr[lev][i + 1] - ls.near_ptr[lev][i])) / 6.0;
  f[4] = std::log2(1.0 + (double)(ls.far_ptr[lev][i + 1] - ls.far_ptr[lev][i])) / 6.0;
  f[5] = std::log2(1.0 + ntargets) / 8.0;
  f[6] = std::log2(1.0 + (double)ncols) / 20.0;
  f[7] = p.tol > 0 ? -std::log10(p.tol) / 16.0 : 1.0;
  f[8] = p.kernel == H2ULV_YUKAWA ? p.alpha * r : 0.0;
  for (int d = 0; d < 3; ++d) f[9 + d] = r > 0 ? std::sqrt(std::max(ev[d], 0.0)) / r : 0.0;
  f[12] = r0 > 0 ? std::log2(std::max(r / r0, std::ldexp(1.0, -30))) / 16.0 : 0.0;
  f[13] = child_ratio;
  f[14] = lev == T.L ? 1.0 : 0.0;
  f[15] = p.eta / 2.0;
  for (int d = 0; d < 16; ++d) out[d] = (float)f[d];
}

h2ulv_rankmodel* rankmodel_create(uint64_t seed) {
  auto M = std::make_unique<h2ulv_rankmodel>();
  std::vector<float> th(MLP_NPARAM, 0.0f);
  const uint64_t key = sketch_key(seed, 0, 0);
  struct Block {
    int off, size, fan_in;
    double gain;
  };
  // weights He-normal (gain 2 / fan-in), output weights 1 / fan-in, biases 0
  const Block blocks[4] = {{MLP_OFF_W1, MLP_W * MLP_NF, MLP_NF, 2.0},
                           {MLP_OFF_W2, MLP_W * MLP_W, MLP_W, 2.0},
                           {MLP_OFF_W3, MLP_W * MLP_W, MLP_W, 2.0},
                           {MLP_OFF_W4, MLP_W, MLP_W, 1.0}};
  for (const Block& b : blocks) {
    const double sc = std::sqrt(b.gain / b.fan_in);
    for (int j = 0; j < b.size; ++j) th[b.off + j] = (float)(host_gauss(key, b.off + j) * sc);
  }
  M->theta.alloc(MLP_NPARAM * sizeof(float));
  M->m.alloc(MLP_NPARAM * sizeof(float));
  M->v.alloc(MLP_NPARAM * sizeof(float));
  H2ULV_HIP(hipMemcpy(M->theta.p, th.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  H2ULV_HIP(hipMemset(M->m.p, 0, MLP_NPARAM * sizeof(float)));
  H2ULV_HIP(hipMemset(M->v.p, 0, MLP_NPARAM * sizeof(float)));
  return M.release();
}

void rankmodel_gradient(const h2ulv_rankmodel& M, const float* feat, const float* target,
                        int64_t n, float* grad, float* loss_host, hipStream_t s) {
  const int64_t nblk = (n + MLP_TILE - 1) / MLP_TILE;
  DBuf part(nblk * MLP_NPARAM * sizeof(float)), pl(nblk * sizeof(float)), lo(sizeof(float));
  launch_mlp_grad(M.theta.as<float>(), feat, target, n, part.as<float>(), pl.as<float>(), s);
  launch_mlp_reduce(part.as<float>(), pl.as<float>(), nblk, grad, lo.as<float>(), s);
  H2ULV_HIP(hipGetLastError());
  float h = 0.0f;
  H2ULV_HIP(hipMemcpyAsync(&h, lo.p, sizeof(float), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  if (loss_host) *loss_host = h;
}

void rankmodel_adam(h2ulv_rankmodel& M, const float* grad, float lr, hipStream_t s) {
  M.step += 1;
  const double bc1 = 1.0 - std::pow(0.9, (double)M.step);
  const double bc2 = 1.0 - std::pow(0.999, (double)M.step);
  launch_adam(M.theta.as<float>(), M.m.as<float>(), M.v.as<float>(), grad, MLP_NPARAM, lr, 0.9f,
              0.999f, 1e-8f, (float)bc1, (float)bc2, s);
  H2ULV_HIP(hipGetLastError());
}

void rankmodel_train(h2ulv_rankmodel& M, const float* feat, const float* target, int64_t n,
                     int steps, float lr, float* loss_host, hipStream_t s) {
  const int64_t nblk = (n + MLP_TILE - 1) / MLP_TILE;
  DBuf part(nblk * MLP_NPARAM * sizeof(float)), pl(nblk * sizeof(float)), lo(sizeof(float)),
      g(MLP_NPARAM * sizeof(float));
  for (int t = 0; t < steps; ++t) {
    launch_mlp_grad(M.theta.as<float>(), feat, target, n, part.as<float>(), pl.as<float>(), s);
    launch_mlp_reduce(part.as<float>(), pl.as<float>(), nblk, g.as<float>(), lo.as<float>(), s);
    rankmodel_adam(M, g.as<float>(), lr, s);
  }
  H2ULV_HIP(hipGetLastError());
  float h = 0.0f;
  H2ULV_HIP(hipMemcpyAsync(&h, lo.p, sizeof(float), hipMemcpyDeviceToHost, s));
  H2ULV_HIP(hipStreamSynchronize(s));
  if (loss_host) *loss_host = h;
}

}  // namespace h2ulv
