// The large-node path (bt_wave.hpp) and the per-lane path (bt_device.hpp)
// built for the CPU, with a wavefront of any width emulated lane by lane
// (BT_HOST_DEBUG), driving whole trees level by level.  Used by the CPU tests
// to compare the cooperative path with the oracle without a GPU.
//
// stdin, one option per line: S0 K K2 R sigma T k N payoff flags
// argv[1] = per-lane threshold (nodes whose children hold more points go to
// the cooperative path; 0 sends every node there), argv[2] = 1 for tangents,
// argv[3] = emulated lanes, argv[4] = 1 to run the envelope's final merge in
// two halves as a helper wave would (binary64).
// stdout, one line per option: error ask bid total_bp_ask total_bp_bid
// max_bp_ask max_bp_bid [8 tangents], numbers in hexadecimal floating point.
#define BT_HOST_DEBUG 1
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "bt_device.hpp"
#include "bt_wave.hpp"
using namespace bt;
template <typename T> T *lds_buf() { static std::vector<T> b(40000); return b.data(); }

template <typename T> struct Rec { std::vector<T> d; int m; };

template <typename T>
static int run_side(const Model& md, int side, T* root, long long* tot, int* mx, int thr) {
  const Inputs<T> in = inputs_of(md, T{});
  int N = md.N;
  std::vector<T> Stab(2*N+3);
  for (int idx = 0; idx < 2*N+3; idx++) Stab[idx] = stock_at(in, idx-(N+1));
  std::vector<Rec<T>> cur(N+2), nxt(N+2);
  const T one = mk<T>(1.0);
  for (int c = 0; c <= N+1; c++) { T S = Stab[2*c]; T Sa=(one+in.k)*S, Sb=(one-in.k)*S; cur[c].d = {-Sa, mk<T>(0.0), mk<T>(0.0), -Sb}; cur[c].m = 1; }
  std::vector<T> tmp;
  static std::vector<double> pool(1 << 25);
  *tot = 0; *mx = 0;
  for (int t = N; t >= 0; t--) {
    T kt = (t >= 1 || (md.flags & F_COST_AT_T0)) ? in.k : mk<T>(0.0);
    bool exercise = !((md.flags & F_EUROPEAN) && t < N);
    for (int c = 0; c <= t; c++) {
      View<T> Zd{cur[c].d.data()+1, cur[c].d.data()+2, cur[c].d.data(), cur[c].m, 3};
      View<T> Zu{cur[c+1].d.data()+1, cur[c+1].d.data()+2, cur[c+1].d.data(), cur[c+1].m, 3};
      int M = cur[c].m + cur[c+1].m;
      T S = Stab[2*c - t + N + 1], xi, ze; payoff(md, in, S, xi, ze);
      Arr<T> Z; int mz = -1;
      if (M <= thr) {
        Caps cp = small_caps();
        tmp.assign(cp.total + 8, mk<T>(NAN));
        mz = side == 0 ? node_update<0, T>(Zu, Zd, S, kt, in.rho, xi, ze, exercise, tmp.data(), 1, cp, &Z)
                       : node_update<1, T>(Zu, Zd, S, kt, in.rho, xi, ze, exercise, tmp.data(), 1, cp, &Z);
      }
      if (mz < 0) {
        WaveTmp W{pool.data(), (int64_t)pool.size(), 0};
        mz = side == 0 ? wave_node_update<0, T>(Zu, Zd, S, kt, in.rho, xi, ze, exercise, W, lds_buf<T>(), &Z)
                       : wave_node_update<1, T>(Zu, Zd, S, kt, in.rho, xi, ze, exercise, W, lds_buf<T>(), &Z);
      }
      if (mz < 0) return -1;
      nxt[c].m = mz; nxt[c].d.resize(3*mz+1);
      nxt[c].d[0] = Z.S(0);
      for (int j = 0; j < mz; j++) { nxt[c].d[1+3*j] = Z.X(j); nxt[c].d[2+3*j] = Z.V(j); nxt[c].d[3+3*j] = Z.S(j+1); }
      int bp = (mz == 1 && val(Z.S(0)) == val(Z.S(1))) ? 0 : mz;
      *tot += bp; if (bp > *mx) *mx = bp;
    }
    std::swap(cur, nxt);
  }
  View<T> z0{cur[0].d.data()+1, cur[0].d.data()+2, cur[0].d.data(), cur[0].m, 3};
  *root = eval(z0, mk<T>(0.0));
  return 0;
}

int main(int argc, char** argv) {
  double S0,K,K2,R,sig,T,k; int N, pay; unsigned fl;
  int thr = argc > 1 ? atoi(argv[1]) : 12;
  int grad = argc > 2 ? atoi(argv[2]) : 0;
  if (argc > 3) bt_host_lanes = atoi(argv[3]);
  if (argc > 4) bt_host_split = atoi(argv[4]);
  while (scanf("%lf %lf %lf %lf %lf %lf %lf %d %d %u", &S0,&K,&K2,&R,&sig,&T,&k,&N,&pay,&fl) == 10) {
    bt_params p{S0, K, K2, R, sig, T, k, N, pay, fl, 0u};
    Model m{};
    if (!derive_model(p, BT_MAX_N, m)) { printf("-1\n"); fflush(stdout); continue; }
    long long ta, tb; int ma, mb;
    if (!grad) {
      double ra, rb;
      int e1 = run_side<double>(m, 0, &ra, &ta, &ma, thr), e2 = run_side<double>(m, 1, &rb, &tb, &mb, thr);
      printf("%d %a %a %lld %lld %d %d\n", e1|e2, ra, -rb, ta, tb, ma, mb);
    } else {
      D4 ra, rb;
      int e1 = run_side<D4>(m, 0, &ra, &ta, &ma, thr), e2 = run_side<D4>(m, 1, &rb, &tb, &mb, thr);
      printf("%d %a %a %lld %lld %d %d %a %a %a %a %a %a %a %a\n", e1|e2, ra.v, -rb.v, ta, tb, ma, mb,
             ra.d[0], ra.d[1], ra.d[2], ra.d[3], -rb.d[0], -rb.d[1], -rb.d[2], -rb.d[3]);
    }
    fflush(stdout);
  }
  fprintf(stderr, "envelope merges: scheduled %lld, walked %lld\n", bt_host_env_sched[0], bt_host_env_sched[1]);
  fprintf(stderr, "split merges: %lld, dropped %lld\n", bt_host_split_stats[0], bt_host_split_stats[1]);
}
