// Host-side exercise of the C ABI for the sanitizer build (address and
// undefined-behaviour checks of the host code): every validation path of
// qoc_create, the (p, n) rule, the status strings and the argument checks
// of the other entry points, without a GPU (a valid problem then stops at
// the device check; with a GPU it is created and destroyed).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/qoc.h"

static int failures = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::printf("FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond,    \
                  qoc_last_error());                                      \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

int main() {
  const int d = 5, M = 2, N = 7, S = 2;
  std::vector<double> H0(2 * d * d, 0.0), Hk(2 * M * d * d, 0.0), psi0(2 * S * d, 0.0),
      psiT(2 * S * d, 0.0), w(d, 0.5), forb(2 * d, 0.0);
  for (int m = 0; m < d; ++m) H0[2 * (m * d + m)] = 0.1 * m;
  for (int k = 0; k < M; ++k)
    for (int m = 0; m + 1 < d; ++m) {  // Hermitian: real symmetric off-diagonals
      Hk[2 * (k * d * d + m * d + m + 1)] = 1.0;
      Hk[2 * (k * d * d + (m + 1) * d + m)] = 1.0;
    }
  psi0[0] = 1.0;
  psi0[2 * (d + 1)] = 1.0;
  psiT[2 * 1] = 1.0;
  psiT[2 * (d + 0)] = 1.0;
  forb[2 * (d - 1)] = 1.0;
  qoc_problem_desc D;
  std::memset(&D, 0, sizeof(D));
  D.d = d; D.M = M; D.N = N; D.S = S; D.dt = 0.1;
  D.H0 = H0.data(); D.Hk = Hk.data(); D.psi0 = psi0.data(); D.psiT = psiT.data();
  D.penalty_w = w.data(); D.alpha_fid = 1.0; D.alpha_pen = 0.1;
  D.n_forbidden = 1; D.forbidden = forb.data(); D.alpha_time = 0.2;
  qoc_handle *h = nullptr;

  // status strings and version
  for (int s = -8; s <= 0; ++s) EXPECT(qoc_status_string((qoc_status)s) != nullptr);
  EXPECT(std::strlen(qoc_version()) > 0);
  // (p, n) rule
  int p = 0, n = 0;
  EXPECT(qoc_taylor_select(0.37, 1e-10, &p, &n) == QOC_OK && p >= 2);
  EXPECT(qoc_taylor_select(-1.0, 1e-10, &p, &n) == QOC_ERR_ARG);
  EXPECT(qoc_taylor_select(NAN, 1e-10, &p, &n) == QOC_ERR_ARG);
  EXPECT(qoc_taylor_select(1.0, 0.0, &p, &n) == QOC_ERR_ARG);
  EXPECT(qoc_taylor_select(1.0, 1e-10, nullptr, &n) == QOC_ERR_ARG);
  for (int form = 0; form < 3; ++form) {
    EXPECT(qoc_select_pair(0.81, 1e-10, form, &p, &n) == QOC_OK && p >= 2 && n >= 0);
    EXPECT(qoc_select_pair(-1.0, 1e-10, form, &p, &n) == QOC_ERR_ARG);
  }
  EXPECT(qoc_select_pair(0.81, 1e-10, QOC_FORM_BATCHED, &p, &n) == QOC_OK && p == 9 && n == 1);
  EXPECT(qoc_select_pair(1.0, 1e-10, 7, &p, &n) == QOC_ERR_ARG);
  EXPECT(qoc_pair_for(nullptr, 1.0, &p, &n) == QOC_ERR_ARG);
  // invalid descriptors
  EXPECT(qoc_create(nullptr, &h) == QOC_ERR_ARG);
  EXPECT(qoc_create(&D, nullptr) == QOC_ERR_ARG);
  auto expect_create = [&](qoc_problem_desc X, qoc_status want) {
    qoc_handle *hh = nullptr;
    const qoc_status s = qoc_create(&X, &hh);
    EXPECT(s == want);
    EXPECT(hh == nullptr);
    if (hh) qoc_destroy(hh);
  };
  { auto X = D; X.d = 0; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.d = 2000; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.S = d + 1; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.M = -1; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.N = 0; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.dt = 0.0; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.H0 = nullptr; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.fid_mode = 3; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.precision = 9; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.checkpoint_every = -2; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.taylor_p = 1; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.pad_multiple = 48; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.segment_steps = -1; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.propagation = 2; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.propagation = QOC_PROP_ACTION; X.precision = QOC_BF16X3;
    expect_create(X, QOC_ERR_UNSUPPORTED); }
  { auto X = D; X.n_forbidden = 17; expect_create(X, QOC_ERR_SHAPE); }
  { auto X = D; X.forbidden = nullptr; expect_create(X, QOC_ERR_ARG); }
  { auto X = D; X.alpha_time = INFINITY; expect_create(X, QOC_ERR_NONFINITE); }
  {
    auto bad = H0;
    bad[3] = NAN;
    auto X = D; X.H0 = bad.data(); expect_create(X, QOC_ERR_NONFINITE);
  }
  {
    auto bad = Hk;
    bad[2 * 1] = 0.7;  // H_1[0][1] != conj(H_1[1][0])
    auto X = D; X.Hk = bad.data(); expect_create(X, QOC_ERR_NOT_HERMITIAN);
  }
  {
    auto bw = w;
    bw[2] = -1.0;
    auto X = D; X.penalty_w = bw.data(); expect_create(X, QOC_ERR_ARG);
  }
  // a valid problem: created on a GPU machine, QOC_ERR_DEVICE without one
  const qoc_status s = qoc_create(&D, &h);
  EXPECT(s == QOC_OK || s == QOC_ERR_DEVICE);
  if (s == QOC_OK) {
    qoc_info info;
    EXPECT(qoc_get_info(h, &info) == QOC_OK);
    EXPECT(qoc_set_bf16x3(h, 16) == QOC_ERR_ARG);
    EXPECT(qoc_set_unitarity_check(h, -1) == QOC_ERR_ARG);
    EXPECT(qoc_set_gradient(h, 7) == QOC_ERR_ARG);
    qoc_destroy(h);
  }
  // NULL handles and invalid arguments of the other entry points
  EXPECT(qoc_forward(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == QOC_ERR_ARG);
  EXPECT(qoc_cost_grad(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         QOC_ERR_ARG);
  EXPECT(qoc_cost_grad_device(nullptr, nullptr, nullptr, nullptr, nullptr) == QOC_ERR_ARG);
  EXPECT(qoc_cost_grad_device_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr) ==
         QOC_ERR_ARG);
  EXPECT(qoc_cost_grad_batched(-1, nullptr, nullptr, nullptr, nullptr, nullptr) == QOC_ERR_ARG);
  EXPECT(qoc_cost_grad_batched(0, nullptr, nullptr, nullptr, nullptr, nullptr) == QOC_OK);
  EXPECT(qoc_get_info(nullptr, nullptr) == QOC_ERR_ARG);
  EXPECT(qoc_set_taylor(nullptr, 8, 1) == QOC_ERR_ARG);
  EXPECT(qoc_set_sweep(nullptr, 0, 1) == QOC_ERR_ARG);
  EXPECT(qoc_set_bf16x3(nullptr, 1) == QOC_ERR_ARG);
  EXPECT(qoc_set_structure(nullptr, 0) == QOC_ERR_ARG);
  EXPECT(qoc_set_unitarity_check(nullptr, 1) == QOC_ERR_ARG);
  EXPECT(qoc_set_gradient(nullptr, 0) == QOC_ERR_ARG);
  EXPECT(qoc_profile_enable(nullptr, 1) == QOC_ERR_ARG);
  EXPECT(qoc_profile_read(nullptr, nullptr, nullptr, 0) == QOC_ERR_ARG);
  double x = 0.0;
  EXPECT(qoc_adam_step(-1, &x, &x, &x, &x, &x, 0.1, 0.9, 0.99, 1e-8, nullptr) == QOC_ERR_ARG);
  EXPECT(qoc_adam_step(1, &x, &x, &x, &x, &x, 0.1, 1.0, 0.99, 1e-8, nullptr) == QOC_ERR_ARG);
  qoc_destroy(nullptr);
  std::printf(failures ? "abi driver: %d failures\n" : "abi driver: ok\n", failures);
  return failures ? 1 : 0;
}
