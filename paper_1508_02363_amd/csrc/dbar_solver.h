// Internal host structures of the D-bar solver (workspace, operator pipeline, per-entry GMRES record).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "dbar.h"
#include "dbar_launch.h"

namespace dbar {

constexpr int kMaxRestart = 64;
// Gram-Schmidt window of the fused x-space step set by dbar_default_opts (0: full orthogonalisation).  Against the
// last two vectors the Krylov cycles of an N = 1024, 16-k Gaussian-potential batch run 0-4 more steps than fully
// orthogonalised ones but read far fewer basis vectors: 12% less time per mixed solve, 22% per FP64 solve; windows
// of 3, 4, 6 and 8 fall in between.
constexpr int kDefaultOrthWindow = 2;

int fail(int code, const std::string& msg);
extern thread_local std::string g_last_error;  // the calling thread's last message (dbar_last_error)

// Owning device allocation that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      if (p) (void)hipFree(p);
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf();
  int ensure(size_t nbytes);
};

// Pinned host allocation (device-to-host flag reads are DMA transfers, not staging kernels).
struct PinnedInts {
  int* p = nullptr;
  size_t count = 0;
  PinnedInts() = default;
  PinnedInts(const PinnedInts&) = delete;
  PinnedInts& operator=(const PinnedInts&) = delete;
  PinnedInts(PinnedInts&& o) noexcept : p(o.p), count(o.count) { o.p = nullptr; o.count = 0; }
  PinnedInts& operator=(PinnedInts&& o) noexcept {
    std::swap(p, o.p);
    std::swap(count, o.count);
    return *this;
  }
  ~PinnedInts();
  int ensure(size_t n);
  int& operator[](size_t i) { return p[i]; }
  int* data() { return p; }
};

struct Twiddles {
  DevBuf d64, d32;  // exp(-2 pi i j / N), j < N
};

// Per batch entry GMRES record (FP64).  H is column-major: H[j * (kMaxRestart + 1) + i].
struct Ctl {
  double sigma[kMaxRestart + 1];   // 1 / ||v_i|| of the unnormalised basis vectors
  double hsum[kMaxRestart + 1];    // sigma_i <v_i, A v_j> summed over Gram-Schmidt passes
  double coef[kMaxRestart + 1];    // update coefficients (Gram-Schmidt, then the solution update)
  double H[kMaxRestart * (kMaxRestart + 1)];
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1];
  double bnorm, rnorm, thresh, resid;
  // condition estimate: sigma_max / sigma_min of the triangular factor of the longest cycle's Hessenberg matrix so far
  // (kappa_n: that cycle's length; both cleared when the entry's solve starts)
  double kappa;
  int jn, iters, cycles, kappa_n;
};

struct EntryResult {
  int iters, cycles;
  double bnorm, rnorm;
  c64 s00;
  c64 hsh;  // iterated method: h at the shift offset, h(2i conj k)
  double kappa;
};

struct BatchCfg {
  int use_graph = 0;
  int method = 0;  // 0: plain (Section 4), 1: iterated (Section 5.3)
  double tol = 1e-12;
  int max_iter = 1000;
  int reorth = 1;
  int check_every = 4;
  double inner_tol = 1e-6;
  int xspace = 0;  // the plain method iterates on s = F^{-1} S
  int orth_window = 0;  // fused x-space step: Gram-Schmidt against the last orth_window vectors (0: all)
};

// Device workspace for a batch of B entries on an N x N grid with restart m.
struct Work {
  ~Work();
  Work() = default;
  Work& operator=(Work&& o) noexcept;
  int N = 0, B = 0, m = 0, prec = 0;
  // captured Krylov step groups -> executable graph; dropped on reallocation.  A captured kernel node keeps its
  // arguments by value, so the key holds everything those arguments depend on besides the workspace pointers:
  // element bytes + method + space, first and end step, reorth + Gram-Schmidt window + window mode, batch B, and the
  // grid (N, M and the bit pattern of L: the transform scales 1/(2 pi L^2), dx^2/2pi and the xi grid are taken from
  // them, and the kernels are specialised for M)
  using GraphKey = std::tuple<int, int, int, int, int, int, uint64_t>;
  std::map<GraphKey, hipGraphExec_t> graphs;
  int graph_epoch = 0;  // tuning epoch the graphs were captured in
  void drop_graphs();
  size_t n = 0;
  size_t Q_bs = 0;
  DevBuf x, bvec, T64, r64, T32, V, Q64, Q32, ex, ey, ex32, ey32, coefG, dmom, dmom32, part_mom, part_vec, part_norm,
      dred, nred, ctl, act, live, kvals, results, shv, unit, unit32, Hbuf;
  DevBuf Sx, mx;  // x-space solves: S = F x and m = h(S) of the last residual evaluation (FP64)
  DevBuf Fx, Ax;  // x-space iterated solves: f = H(h) and the shifted inverse of h of the last residual evaluation
  // Where an x-space solve leaves S and m: the caller's device arrays when it passes them (set per batch), else null
  // (then Sx / mx, or Fx for the iterated method's S, and the caller gets a copy)
  void* outS = nullptr;
  void* outm = nullptr;
  // x holds zero without having been written: the next solution update (fused into the residual's first launch)
  // writes x = sum y_i V_i instead of adding to it
  bool x_zero = false;
  // Per entry: a windowed Krylov cycle ended it at the restart length rather than at its threshold (strong potentials
  // stall under truncated orthogonalisation), so its later cycles orthogonalise against every basis vector.  The
  // device flags are act[2B + b] (set by the cycle start from the restart flags act[B + b], cleared when the entry's
  // solve starts); this host mirror, updated from the flags the host reads anyway, tells whether a cycle's launches
  // must cover the whole basis.  Other entries keep their window inside such launches.
  std::vector<int> full_host;
  void* S_dst(int method) { return outS ? outS : method == 1 ? Fx.p : Sx.p; }
  void* m_dst() { return outm ? outm : mx.p; }
  PinnedInts host_act, host_live;
  int setup(int N_, int B_, int m_, int prec_, bool shared_q);
  size_t vec_bytes(int prec) const;
};

// The operator pipeline for one grid (pointers into a Work).
constexpr unsigned kShifted = 1u;    // regularise about xi = a = 2i conj(k) (Section 5.1, equation dbarinvShift)
constexpr unsigned kUnitPhase = 2u;  // k = 0 phase (the operator K0 of equation shift)
// Y argument of the x-space operator standing for its right-hand side -i q_k (q_k as the operator's phase flags give
// it): the last launch forms it from the q_k it reads anyway, so a residual b - A(x) reads no b array
inline const void* const kYRhs = reinterpret_cast<const void*>(static_cast<uintptr_t>(1));

// Gram-Schmidt products fused into the operator's last kernel: Re<V_i, out> for i < nv as per-tile partials
// Extra outputs of the x-space operator: S = F s and h(S) of the input (strides n), and the result rounded to FP32
// (r32, stride r32_bs; with out = null the FP64 result itself is not stored).  Any may be null.
struct XOut {
  void* S = nullptr;
  void* h = nullptr;
  void* r32 = nullptr;
  size_t r32_bs = 0;
};

// Extra outputs of the x-space iterated operator (Section 5.3; ξ-space arrays except ha and h0, strides n): h = F eta,
// f = H(h), ha = the shifted regularised inverse of h, h0 = h(f); r32 as in XOut.  Any may be null.
struct XOutB {
  void* hxi = nullptr;
  void* f = nullptr;
  void* ha = nullptr;
  void* h0 = nullptr;
  void* r32 = nullptr;
  size_t r32_bs = 0;
};

// A pending classical Gram-Schmidt update folded into the x-space operator's first launch (see apply_x_first).
struct UpdReq {
  const void* V = nullptr;
  size_t V_bs = 0;
  int nv = 0;
  const double* coef = nullptr;
  int coef_bs = 0;
  double* part = nullptr;  // |v|^2 partials [b][row tile] (null: none)
  double sign = 1.0;       // in -= sign sum coef_i V_i
  bool v32 = false;        // V in FP32 (FP64 input)
  bool zero_in = false;    // the input counts as zero (never read): in = -sign sum coef_i V_i
  // with ctl set, the launch that reduces the moments also takes the Givens step of Krylov step j (restart m) from the
  // |v|^2 partials in part
  Ctl* ctl = nullptr;
  int j = 0, m = 0;
};

struct DotReq {
  const void* V = nullptr;
  size_t V_bs = 0;
  int nv = 0;
  double* part = nullptr;
  bool self = false;  // x-space: |out|^2 too, as value nv (nv + 1 values per entry)
  const int* full = nullptr;  // per-entry window (x-space): entries with full[b] == 0 skip the first `skip` vectors
  int skip = 0;
};

struct Pipeline {
  int N = 0, M = 11;
  double L = 1.0;
  size_t n = 0;
  const void* tw64 = nullptr;  // exp(-2 pi i j / N), j < N, in FP64 and rounded to FP32
  const void* tw32 = nullptr;
  const c64* ex = nullptr;
  const c64* ey = nullptr;
  const c32* ex32 = nullptr;
  const c32* ey32 = nullptr;
  const c64* unit = nullptr;
  const c32* unit32 = nullptr;
  const int* shv = nullptr;
  c64* coefG = nullptr;
  c64* dmom = nullptr;
  c32* dmom32 = nullptr;
  double* part_mom = nullptr;
  double* part_vec = nullptr;
  // apply / rhs act on s = F^{-1} S (the plain method's x-space form) instead of S
  bool xspace = false;

  LineArgs base(int B, const int* act, unsigned flags) const;
  // tiles (blocks per entry) of the launch whose partials (norms, Gram-Schmidt products) apply leaves
  int apply_tiles(bool fp64) const;
  // blocks per entry of rhs's norm partials
  int rhs_blocks() const;
  template <typename T>
  void moments(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, unsigned flags, hipStream_t s) const;
  template <typename T>
  void apply_impl(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
                  int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs, bool want_norm,
                  unsigned flags, const void* S_ep, size_t S_ep_bs, hipStream_t s, const DotReq* dr = nullptr) const;
  // A(S) of the plain method (Section 4), as alpha S + beta i F(q_k conj(h(S))) + gamma Y; in x-space (xspace) the
  // same on s = F^{-1} S, with the extra outputs xo names (may be null)
  template <typename T>
  void apply(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf, int B,
             const int* act, double alpha, double beta, const void* Y, size_t Y_bs, bool want_norm,
             hipStream_t s, const DotReq* dr = nullptr, const XOut* xo = nullptr) const;
  // H(h) of equation eqh2
  template <typename T>
  void H_of(const void* in, size_t in_bs, void* Hout, size_t H_bs, const void* Qp, size_t Q_bs, void* Tbuf, int B,
            const int* act, hipStream_t s) const;
  // B(h) = h - K0(H(h)) of equation eqh2, as alpha h + beta i F(Q conj(F^{-1}(H/xi))) + gamma Y
  template <typename T>
  // In x-space (xspace) the same on eta = F^{-1} h: eta + i q conj(h0(F psi)) with psi = F^{-1} H(F eta) in Hbuf.
  void apply_B(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
               void* Hbuf, int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs,
               bool want_norm, hipStream_t s, const DotReq* dr = nullptr, const XOutB* xb = nullptr) const;
  // x-space B in two parts as apply_x_first / apply_x_rest: the first launch of the shifted pass and its moment
  // reduction (with u: the pending update of the input first), then the rest of both passes
  template <typename T>
  void apply_B_first(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, const UpdReq* u,
                     hipStream_t s) const;
  template <typename T>
  void apply_B_rest(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
                    void* Hbuf, int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs,
                    bool want_norm, hipStream_t s, const DotReq* dr, const XOutB* xb) const;
  void rhs(const void* Q64p, size_t Q_bs, void* T64, c64* bout, int B, const int* act, unsigned flags,
           hipStream_t s) const;
  // x-space: -i q_k straight into out (stride out_bs; FP32 if out32, the first basis vector of a mixed solve), with
  // the |.|^2 partials of its FP64 values (rhs_blocks() per entry)
  void rhs_x(const void* Q64p, size_t Q_bs, void* out, size_t out_bs, bool out32, int B, const int* act,
             unsigned flags, hipStream_t s) const;
  template <typename T>
  void h_of(const void* in, size_t in_bs, void* hout, size_t hout_bs, void* Tbuf, int B, const int* act,
            hipStream_t s, unsigned flags = 0u, bool phase_out = false, bool accumulate = false) const;
  template <typename T>
  void transform(bool inverse, const void* in, void* out, void* Tbuf, hipStream_t s) const;
  // x-space operator: F^{-1} A(F s) = alpha s + beta i q_k conj(h(F s)) + gamma Y (three line launches)
  // The same in two parts: the first launch and the moment reduction (with u, in -= sum coef_i V_i first, written back
  // in place), then the division, the inverse transform and the result (which expects the first part's Tbuf and
  // moments).
  template <typename T>
  void apply_x_first(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, unsigned flags,
                     const UpdReq* u, hipStream_t s) const;
  template <typename T>
  void apply_x_rest(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
                    int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs, bool want_norm,
                    hipStream_t s, const DotReq* dr, const XOut* xo, unsigned flags, const void* S_ep,
                    size_t S_ep_bs) const;
  // flags: kShifted / kUnitPhase as in base(); S_ep: the alpha term's vector (null: the input)
  template <typename T>
  void apply_x(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
               int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs, bool want_norm,
               hipStream_t s, const DotReq* dr, const XOut* xo, unsigned flags = 0u, const void* S_ep = nullptr,
               size_t S_ep_bs = 0) const;
};

void launch_roll_add(const c64* f, const c64* h, const int* shv, int N, c64* out, int B, hipStream_t s);
void launch_add_phase(c64* m, const c64* ha, const c64* ex, const c64* ey, int N, int B, hipStream_t s);

int validate_grid(const dbar_grid* g);
// batched solve behind dbar_solve / dbar_solve_device; r_out (host, nk complex or NULL) receives i h(2i conj k) of
// the iterated method, and with S = m = NULL only that is formed
int solve_impl(const dbar_grid* grid, const void* Q, bool q_on_device, int64_t nk, const double* k, double tol,
               const dbar_opts* opts_in, void* S, void* m, bool out_on_device, dbar_info* info, hipStream_t caller,
               double* r_out);
// Device twiddles of length N from the library's cache (created on first use; the pointers are read under the cache's
// lock).  dbar_release() frees the cache: holders of these pointers across calls must keep copies of their own.
int get_twiddles(int N, const void** d64, const void** d32);
// exp(-2 pi i j / N), j < N, evaluated in long double and rounded once to FP64 and to FP32 (host arrays of N each)
void host_twiddles(int N, c64* out64, c32* out32);
int make_pipeline(const dbar_grid* g, Work& w, Pipeline* p);
// e_k tables of B entries: FP64 ex/ey and their FP32 roundings ex32/ey32 (per-entry stride N)
void launch_phase_tables(const c64* kv_dev, int N, double L, c64* ex, c64* ey, c32* ex32, c32* ey32, int B,
                         hipStream_t s);
int run_batch(const Pipeline& P, Work& w, const BatchCfg& cfg, hipStream_t s, std::vector<int>& iters_out);
// x-space: the residual evaluation's outputs (w.Sx, w.mx; with iterated also w.Fx, w.Ax) = 0 for entries that are
// not live (and in mask, if given): those no residual evaluation writes
void launch_zero_done(Work& w, const int* mask, bool iterated, hipStream_t s);
int ctl_blocks(int B);
// one lockstep Krylov cycle over the entries flagged in w.act; returns the iterations run
template <typename T>
int krylov_cycle(const Pipeline& P, Work& w, const BatchCfg& cfg, int it_budget, hipStream_t s);
// solution update from the cycle and the FP64 residual r = b - A(x) into r_out (norms into w.nred); cond: also the
// condition estimate of the entries whose cycle was their longest so far; outputs (x-space): also the solve's outputs
// if this evaluation is the last (S = F x and m = h(S), or the iterated method's h, f, the shifted inverse and h(f));
// false: the caller knows it is not the last
template <typename T>
void end_cycle(const Pipeline& P, Work& w, int nv, void* r_out, hipStream_t s, int method = 0, bool cond = true,
               bool outputs = true);
// condition estimate of each live entry from its last cycle's Hessenberg factor, where that cycle is the longest so far
void launch_cond_estimate(Work& w, hipStream_t s);
// residual check (first = 1: record ||b|| and reset the counters of the entries in mask); tolv: per-entry tol
void launch_ctl_check(Work& w, double tol, int first, const int* mask, const double* tolv, hipStream_t s);
// start a cycle for every live entry from its residual norm
void launch_ctl_start(Work& w, double abs_tol, double rel_tol, const double* tolv, hipStream_t s);

}  // namespace dbar
