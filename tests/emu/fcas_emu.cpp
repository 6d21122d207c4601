// CPU emulator of one fitness evaluation through the library's own tile and
// stage functions (paper_2002_02150_amd/csrc/fitness_tiles.hpp), thread by
// thread, with a separate LDS buffer per transform and the kernel's
// write / barrier / read order.  Built with the host address sanitizer by the
// tests, so any out-of-range index in the pass logic aborts on the CPU.
//
// usage: fcas_emu <precision 0|1> <plan> <n_det> <k_lo> <k_hi> <df> <f_star> <in_prefix> <out_file>
//   inputs  <in_prefix>.{pos,ten,sigma,b,theta} float64, <in_prefix>.y complex64 or complex128 [K][n_det]
//   output  N float64 Gamma^2_j, then best value, best sample (float64)
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plans.hpp"

using namespace fcas;

template <typename T>
static std::vector<T> read_all(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) { std::perror(path.c_str()); std::exit(2); }
  std::fseek(f, 0, SEEK_END);
  long bytes = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<T> v(bytes / sizeof(T));
  if (std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) std::exit(3);
  std::fclose(f);
  return v;
}

template <typename Real, int E>
struct Regs {
  cplx<Real> v[2][E];
};

// All stages of a length-L transform for `nt` threads sharing one LDS buffer
// per transform: buffer of thread `tid` is bufs[owner(tid)], index t = pos(tid).
template <typename Real, int L, int E, class Rad, int I, int Ns, bool HALF, int PAD, class Owner, class Pos>
static void emu_stages(std::vector<Regs<Real, E>>& regs, std::vector<std::vector<cplx<Real>>>& bufs,
                       const std::vector<cplx<Real>>& tw, Owner owner, Pos pos) {
  if constexpr (I < Rad::count) {
    constexpr int R = Rad::value[I];
    constexpr bool LAST = (I == Rad::count - 1);
    for (int s = 0; s < 2; ++s) {
      for (size_t tid = 0; tid < regs.size(); ++tid)
        stage_butterflies<Real, L, E, R, Ns, LAST, HALF && I == 0, PAD>(regs[tid].v[s], bufs[owner(tid)].data(),
                                                                       tw.data(), pos(tid));
      if constexpr (!LAST) {
        for (size_t tid = 0; tid < regs.size(); ++tid)
          stage_gather<Real, L, E, PAD>(regs[tid].v[s], bufs[owner(tid)].data(), pos(tid));
      }
    }
    emu_stages<Real, L, E, Rad, I + 1, Ns * R, false, PAD>(regs, bufs, tw, owner, pos);
  }
}

template <typename Real, class PL, int DT>
static void prologue(cplx<Real> (&v)[2][PL::E1], const EvalDesc& ev, const SegDesc& sg, int n_det, int tile, int c,
                     int p) {
  if constexpr (DT > 0) {
    Pass1Data<Real, PL, DT> d;
    pass1_fetch<Real, PL, DT>(d, sg, tile, c, p);
    pass1_compute<Real, PL, DT>(v, d, pass1_point<Real, DT>(&ev));
  } else {
    pass1_prologue<Real, PL, 0>(v, ev, sg, n_det, tile, c, p);
  }
}

template <typename Real, class PL, int DT>
static void run(const SegDesc& sg, const EvalDesc& ev, int n_det, std::vector<double>& series, double& bg,
                int& bj) {
  const int64_t N = PL::N;
  std::vector<cplx<Real>> ws(2 * N);
  std::vector<cplx<Real>> tw1(PL::N1), tw2(PL::N2);
  for (int m = 0; m < PL::N1; ++m) tw1[m] = twiddle<Real>(m, PL::N1);
  for (int m = 0; m < PL::N2; ++m) tw2[m] = twiddle<Real>(m, PL::N2);
  const int LP1 = lds_padded_len<kPad1>(PL::N1), LP2 = lds_padded_len<kPad2>(PL::N2);
  for (int tile = 0; tile < PL::TILES1; ++tile) {
    std::vector<Regs<Real, PL::E1>> regs(PL::T1);
    std::vector<std::vector<cplx<Real>>> bufs(PL::C, std::vector<cplx<Real>>(LP1));
    for (int tid = 0; tid < PL::T1; ++tid)
      prologue<Real, PL, DT>(regs[tid].v, ev, sg, n_det, tile, tid % PL::C, tid / PL::C);
    emu_stages<Real, PL::N1, PL::E1, typename PL::Rad1, 0, 1, true, kPad1>(
        regs, bufs, tw1, [](size_t t) { return (int)(t % PL::C); }, [](size_t t) { return (int)(t / PL::C); });
    for (int tid = 0; tid < PL::T1; ++tid) pass1_store<Real, PL>(regs[tid].v, ws.data(), tile, tid % PL::C, tid / PL::C);
  }
  if constexpr (PL::THREE) {
    std::vector<cplx<Real>> twm(PL::NM);
    for (int m = 0; m < PL::NM; ++m) twm[m] = twiddle<Real>(m, PL::NM);
    const int LPM = lds_padded_len<kPadM>(PL::NM);
    for (int tile = 0; tile < PL::N1 * (PL::N2 / PL::CM); ++tile) {
      std::vector<Regs<Real, PL::EM>> regs(PL::TM);
      std::vector<std::vector<cplx<Real>>> bufs(PL::CM, std::vector<cplx<Real>>(LPM));
      for (int tid = 0; tid < PL::TM; ++tid) {
        passm_fetch<Real, PL>(regs[tid].v, ws.data(), tile, tid % PL::CM, tid / PL::CM);
        passm_twiddle_in<Real, PL>(regs[tid].v, tile, tid % PL::CM, tid / PL::CM);
      }
      emu_stages<Real, PL::NM, PL::EM, typename PL::RadM, 0, 1, false, kPadM>(
          regs, bufs, twm, [](size_t t) { return (int)(t % PL::CM); }, [](size_t t) { return (int)(t / PL::CM); });
      for (int tid = 0; tid < PL::TM; ++tid) {
        passm_twiddle_out<Real, PL>(regs[tid].v, tile, tid % PL::CM, tid / PL::CM);
        passm_store<Real, PL>(regs[tid].v, ws.data(), tile, tid % PL::CM, tid / PL::CM);
      }
    }
  }
  series.assign(N, -1.0);
  bg = -1;
  bj = 0x7fffffff;
  for (int tile = 0; tile < PL::TILES2; ++tile) {
    std::vector<Regs<Real, PL::E2>> regs(PL::T2);
    std::vector<std::vector<cplx<Real>>> bufs(PL::RW, std::vector<cplx<Real>>(LP2));
    for (int tid = 0; tid < PL::T2; ++tid)
      pass2_load<Real, PL>(regs[tid].v, ws.data(), tile, tid / PL::P2, tid % PL::P2);
    emu_stages<Real, PL::N2, PL::E2, typename PL::Rad2, 0, 1, false, kPad2>(
        regs, bufs, tw2, [](size_t t) { return (int)(t / PL::P2); }, [](size_t t) { return (int)(t % PL::P2); });
    for (int tid = 0; tid < PL::T2; ++tid) {
      const int r = tid / PL::P2, p = tid % PL::P2;
      const int j0 = row_base<PL>(tile * PL::RW + r);
      for (int q = 0; q < PL::E2; ++q) {
        const int64_t j = j0 + (int64_t)PL::ROWS2 * (p + q * PL::P2);
        if (series.at(j) != -1.0) { std::fprintf(stderr, "sample %lld written twice\n", (long long)j); std::exit(4); }
        series.at(j) = (double)(norm2(regs[tid].v[0][q]) + norm2(regs[tid].v[1][q]));
      }
      Real g;
      int j;
      pass2_best<Real, PL>(regs[tid].v, tile, r, p, g, j);
      if (better((double)g, j, bg, bj)) { bg = (double)g; bj = j; }
    }
  }
  for (int64_t j = 0; j < N; ++j)
    if (series[j] < 0) { std::fprintf(stderr, "sample %lld never written\n", (long long)j); std::exit(5); }
}

template <typename Real>
static int main_t(int plan, int n_det, int k_lo, int k_hi, double df, double f_star, const std::string& in,
                  const std::string& out) {
  auto pos = read_all<double>(in + ".pos");
  auto ten = read_all<double>(in + ".ten");
  auto sig = read_all<double>(in + ".sigma");
  auto b = read_all<double>(in + ".b");
  auto th = read_all<double>(in + ".theta");
  auto y = read_all<cplx<Real>>(in + ".y");
  const int K = k_hi - k_lo + 1;
  if ((int)b.size() != K || (int)y.size() != K * n_det || (int)pos.size() != 3 * n_det) {
    std::fprintf(stderr, "input sizes do not match\n");
    return 6;
  }
  NetDesc net{};
  net.n_det = n_det;
  net.f_star = f_star;
  std::memcpy(net.pos, pos.data(), sizeof(double) * 3 * n_det);
  std::memcpy(net.ten, ten.data(), sizeof(double) * 9 * n_det);
  SegDesc sg{};
  sg.y = y.data();
  sg.b = b.data();
  sg.n = kPlans[plan].n;
  sg.k_lo = k_lo;
  sg.k_hi = k_hi;
  sg.plan = plan;
  sg.registered = 1;
  sg.dk1 = (int32_t)(kPlans[plan].n / kPlans[plan].e1);
  sg.df = df;
  for (int i = 0; i < n_det; ++i) sg.sigma[i] = sig[i];
  EvalDesc ev{};
  setup_one(net, sg, th.data(), ev);
  std::vector<double> series;
  double bg;
  int bj;
#define FCAS_EMU_CASE(id, ...)                                                                         \
  case id: {                                                                                           \
    using PL = std::conditional_t<std::is_same_v<Real, float>, PlanF##id, PlanD##id>;                  \
    if (n_det == 1) run<Real, PL, 1>(sg, ev, n_det, series, bg, bj);                                   \
    else if (n_det == 2) run<Real, PL, 2>(sg, ev, n_det, series, bg, bj);                              \
    else if (n_det == 3) run<Real, PL, 3>(sg, ev, n_det, series, bg, bj);                              \
    else if (n_det == 4) run<Real, PL, 4>(sg, ev, n_det, series, bg, bj);                              \
    else run<Real, PL, 0>(sg, ev, n_det, series, bg, bj);                                              \
    break;                                                                                             \
  }
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_EMU_CASE)
    default:
      return 7;
  }
  FILE* f = std::fopen(out.c_str(), "wb");
  std::fwrite(series.data(), sizeof(double), series.size(), f);
  const double tail[2] = {bg, (double)bj};
  std::fwrite(tail, sizeof(double), 2, f);
  std::fclose(f);
  return 0;
}

// Checks the fused-schedule sequence for cnt evaluations with lag L and S
// slots: every (kind, ep, tile) appears exactly once, a pass-2 tile comes after
// all pass-1 tiles of its evaluation, and a pass-1 tile comes after all pass-2
// tiles of the evaluation that used its slot before (ep - S).
static int check_schedule(int cnt, int L, int S, int T1, int T2) {
  const int total = cnt * (T1 + T2);
  std::vector<int> pos1((size_t)cnt * T1, -1), pos2((size_t)cnt * T2, -1);
  for (int i = 0; i < total; ++i) {
    int kind, ep, tile;
    fused_decode(i, cnt, L, T1, T2, kind, ep, tile);
    if (ep < 0 || ep >= cnt) return 10;
    if (kind == 1) {
      if (tile < 0 || tile >= T1 || pos1.at((size_t)ep * T1 + tile) != -1) return 11;
      pos1[(size_t)ep * T1 + tile] = i;
    } else if (kind == 2) {
      if (tile < 0 || tile >= T2 || pos2.at((size_t)ep * T2 + tile) != -1) return 12;
      pos2[(size_t)ep * T2 + tile] = i;
    } else {
      return 13;
    }
  }
  for (int ep = 0; ep < cnt; ++ep) {
    int last1 = -1, first1 = total, last2 = -1, first2 = total;
    for (int t = 0; t < T1; ++t) {
      last1 = std::max(last1, pos1[(size_t)ep * T1 + t]);
      first1 = std::min(first1, pos1[(size_t)ep * T1 + t]);
    }
    for (int t = 0; t < T2; ++t) first2 = std::min(first2, pos2[(size_t)ep * T2 + t]);
    if (last1 >= first2) return 14;   // pass 2 before its pass 1
    if (ep >= S) {
      for (int t = 0; t < T2; ++t) last2 = std::max(last2, pos2[(size_t)(ep - S) * T2 + t]);
      if (last2 >= first1) return 15;   // slot reused too early
    }
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc == 7 && std::string(argv[1]) == "schedule") {
    return check_schedule(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5]),
                          std::atoi(argv[6]));
  }
  if (argc != 10) {
    std::fprintf(stderr, "usage: %s prec plan n_det k_lo k_hi df f_star in_prefix out\n", argv[0]);
    return 1;
  }
  const int prec = std::atoi(argv[1]), plan = std::atoi(argv[2]), n_det = std::atoi(argv[3]);
  const int k_lo = std::atoi(argv[4]), k_hi = std::atoi(argv[5]);
  const double df = std::atof(argv[6]), f_star = std::atof(argv[7]);
  return prec ? main_t<double>(plan, n_det, k_lo, k_hi, df, f_star, argv[8], argv[9])
              : main_t<float>(plan, n_det, k_lo, k_hi, df, f_star, argv[8], argv[9]);
}
