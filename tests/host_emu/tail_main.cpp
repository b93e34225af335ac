// Driver of the host build of k_spatial_tail (see gen_tail.py): every tail the
// library can launch (n = 2^m - 1 whose sub-levels fit the LDS budget, d = 1..3,
// N_t = 1..4, FP64 and FP32) with nu1x, nu2x in 0..3 and each update mode, three
// slabs, 256 threads per workgroup, LDS and vectors in heap buffers of exactly
// the launch's sizes.
#include "tail_kernel.inc"
using namespace stmg;

template <typename T, int D, int NT>
int run(int n0, int nu1, int nu2, int upd, long long slabs, bool with_base) {
  // sub-levels from n0 down to one node, as the host builds them
  std::vector<int> ns;
  for (int m = n0; m >= 1; m = (m - 1) / 2) { ns.push_back(m); if (m == 1) break; }
  const size_t lds = spatial_tail_lds(D, n0, NT, sizeof(T));
  if (lds == 0 || (int)ns.size() > TAIL_MAX) return 0;
  TailArgs<T> a{};
  for (int i = 0; i < NT * NT; ++i) { a.K[i] = T(0.1) * (i + 1); a.M[i] = T(0.01) * (i + 2); }
  a.levels = (int)ns.size();
  for (int q = 0; q < a.levels; ++q) {
    for (int i = 0; i < NT * NT; ++i) a.Dinv[q][i] = T(0.3) / (1 + i);
    for (int i = 0; i < 3; ++i) { a.wm[q][i] = T(1) / (i + 2); a.wk[q][i] = T(i == 1 ? 2 : -1); }
    a.n[q] = ns[q];
  }
  a.slabs = slabs; a.omega = T(2) / 3; a.upd = upd; a.scale = T(0.5); a.nu1 = nu1; a.nu2 = nu2;
  long long nx0 = 1; for (int i = 0; i < D; ++i) nx0 *= n0;
  const size_t len = (size_t)slabs * NT * nx0;
  T* f = (T*)malloc(len * sizeof(T));
  T* out = (T*)malloc(len * sizeof(T));
  T* base = with_base ? out : nullptr;
  for (size_t i = 0; i < len; ++i) { f[i] = T((i % 17) * 0.1); out[i] = T(1); }
  g_lds = (unsigned char*)malloc(lds);
  memset(g_lds, 0, lds);
  gridDim = {1, (unsigned)slabs, 1};
  blockDim = {256, 1, 1};
  for (unsigned by = 0; by < gridDim.y; ++by)
    for (unsigned t = 0; t < 256; ++t) {
      blockIdx = {0, by, 0};
      threadIdx = {t, 0, 0};
      k_spatial_tail<T, D, NT>(f, base, out, a);
    }
  free(g_lds); free(f); free(out);
  return 1;
}

template <typename T, int D>
int sweep_nt(int n0, int nu1, int nu2, int upd, bool wb) {
  return run<T, D, 1>(n0, nu1, nu2, upd, 3, wb) + run<T, D, 2>(n0, nu1, nu2, upd, 3, wb) +
         run<T, D, 3>(n0, nu1, nu2, upd, 3, wb) + run<T, D, 4>(n0, nu1, nu2, upd, 3, wb);
}

int main() {
  int cases = 0;
  const int ns[] = {1, 3, 7, 15, 31, 63, 127, 255};
  for (int n0 : ns)
    for (int nu1 = 0; nu1 <= 3; ++nu1)
      for (int nu2 = 0; nu2 <= 3; ++nu2)
        for (int upd = 0; upd <= 2; ++upd) {
          const bool wb = upd == UPD_ADD;
          cases += sweep_nt<double, 1>(n0, nu1, nu2, upd, wb) + sweep_nt<double, 2>(n0, nu1, nu2, upd, wb) +
                   sweep_nt<double, 3>(n0, nu1, nu2, upd, wb) + sweep_nt<float, 1>(n0, nu1, nu2, upd, wb) +
                   sweep_nt<float, 2>(n0, nu1, nu2, upd, wb) + sweep_nt<float, 3>(n0, nu1, nu2, upd, wb);
        }
  printf("cases run: %d\n", cases);
  return 0;
}
