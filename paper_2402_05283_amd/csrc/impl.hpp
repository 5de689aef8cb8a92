// Plan state and per-size kernel dispatch of the CPRA library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <string>
#include <vector>

#include "../../include/cpra.h"
#include "host_geom.hpp"
#include "kernels.hpp"
#include "merge.hpp"
#include "shrink.hpp"
#include "refine.hpp"
#include "stepd.hpp"

namespace cpra_impl {

struct Layout {
  size_t P, Pmid, Pc, g0, g1, A2, ampscale, maskw, den, tw, coup, alist, iota, errpart, errhist, flags, stage_I,
      stage_S, csr_ptr, csr_cell, csr_heavy, csr_ent, csr_w, cnt_inv, plane, stage_T, prep_part, mtab, swk, ctab, total;
  int zc;   // z-planes per step-D chunk
};

// Process-wide pool of pinned host buffers.  A plan's staging buffers go back to the pool when it is
// destroyed instead of to hipHostFree, which waits for every stream of the device; pooled buffers
// are held until the process ends.  pinned_take returns nullptr if the allocation fails.
void* pinned_take(size_t bytes);
void pinned_give(void* p, size_t bytes);

}  // namespace cpra_impl

struct cpra_plan_s {
  cpra_params p{};
  int R = 1;                   // guesses (independent reconstructions); slot r * Np + n
  std::vector<double> taps;    // 2K+1 taps of Eq. 4 when K >= 2 (else alpha[3] and the fused path)
  int K = 1;
  std::vector<double> theta;
  cpra_impl::Layout L{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;              // HIP device the plan was created on
  int cur = 0;                 // which g buffer holds the current iterate
  int64_t k = 0;               // global iteration count
  std::vector<uint8_t> landed, present;
  std::vector<int32_t> alist_h;
  bool tables_dirty = true;
  bool poisoned = false;
  std::string err;
  int ntiles = 0;
  std::vector<cpra_host::Coupling> coup_h;
  std::vector<cpra_host::Tap> tap_h;
  std::vector<double> errhist_h;
  // optional per-pass event timing (measurement): triples (before col, between, after row)
  bool timing = false;
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  hipEvent_t next_event() {
    if (ev_used == evpool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      evpool.push_back(e);
    }
    return evpool[ev_used++];
  }
  // HIP graphs of one episode (n_ei iterations from a boundary), one per parity of cur, valid for
  // one angle set (table_version), algorithm and beta
  bool use_graphs = false;
  // slots per chunk of the chunk-major order inside an episode (0: all slots in every launch)
  int chunk = 0;
  // the row pass's tile height: RowCfg's (false) or twice it (true); set by a tuning
  bool row_alt = false;
  // step-D insertion tables: uploaded at the first step-D call from a pinned image that the
  // process caches per shape (ev_stepd: the uploads have completed); h_stepd holds the plan's own
  // image when the cache was full
  bool stepd_ready = false;
  int n_heavy = 0;             // step-D cells summed by a wavefront each
  void* h_stepd = nullptr;
  size_t stepd_bytes = 0;
  hipEvent_t ev_stepd = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_batch = nullptr;   // orders a fused batch's stream and the plan's own stream
  // pinned staging of the coupling tables and slot list: a ring of kTabSlots buffers, so that an
  // upload waits only for the one kTabSlots uploads back (ev_tab[i]: slot i's copies completed)
  static constexpr int kTabSlots = 4;
  void* h_tab = nullptr;
  size_t tab_bytes = 0;
  hipEvent_t ev_tab[kTabSlots] = {};
  bool tab_pending[kTabSlots] = {};
  int tab_next = 0;
  // the data check of asynchronous submits: the device flag copied to pinned memory (ev_flag)
  int32_t* h_flag = nullptr;
  hipEvent_t ev_flag = nullptr;
  bool flag_pending = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int g_algo = -1;
  double g_beta = 0.0;
  uint64_t g_version = 0, table_version = 1;
  void drop_graphs() {
    for (auto& g : gexec) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  }
  int pid = 0;                 // creating process: a forked child must make no HIP call on its copy
  ~cpra_plan_s() {
    if (pid != (int)getpid()) return;
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_batch) (void)hipEventDestroy(ev_batch);
    for (int i = 0; i < kTabSlots; ++i)
      if (tab_pending[i]) (void)hipEventSynchronize(ev_tab[i]);
    if (flag_pending) (void)hipEventSynchronize(ev_flag);
    if (ev_stepd) {
      (void)hipEventSynchronize(ev_stepd);
      (void)hipEventDestroy(ev_stepd);
    }
    for (hipEvent_t ev : ev_tab)
      if (ev) (void)hipEventDestroy(ev);
    if (ev_flag) (void)hipEventDestroy(ev_flag);
    cpra_impl::pinned_give(h_tab, tab_bytes * kTabSlots);
    cpra_impl::pinned_give(h_flag, 256);
    cpra_impl::pinned_give(h_stepd, stepd_bytes);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
  }
};


namespace cpra_impl {
using namespace cpra;

template <typename X> X* at(cpra_plan_t pl, size_t off) { return reinterpret_cast<X*>(pl->ws + off); }

// device buffers and settings of one 3D refinement (the caller's refinement workspace)
struct RefineArgs {
  void* vol;          // N^3 real: the step-D volume in, the refined volume out
  void* qh;           // N^3 complex: measured mixed-domain values (NaN = free)
  void* cb;           // N^3 complex: row spectra of the iterate; blur scratch
  uint8_t* s3;        // N^3 support
  double* pmax;       // blur maxima (N * N / 8 + 1)
  void* win;          // blur window taps (2W + 1)
  const double* sc;   // (sin, cos) per listed angle
  const int* list;    // present data angles
  int count, n_iter, shrink_every, W;
  double threshold;
};

struct Ops {
  void (*twiddles)(cpra_plan_t);
  void (*prep)(cpra_plan_t, const float*, const uint8_t*, int, int);
  void (*init)(cpra_plan_t, const int*, int, int);
  void (*step)(cpra_plan_t, const int*, int, bool, bool, int, double, double*, const void*, int);
  void (*assemble)(cpra_plan_t, void*);
  void (*reload)(cpra_plan_t, const int*, int, int);
  void (*colerr)(cpra_plan_t, const int*, int, double*);
  void (*moments)(cpra_plan_t, const int*, int, double*);
  void (*twin)(cpra_plan_t, const int*, const int*, int, double*);
  void (*merge_avg)(cpra_plan_t, int, const int*, const int*, const int*, void*);
  void (*shrinkwrap)(cpra_plan_t, const int*, int, int, double);
  void (*couple_taps)(cpra_plan_t, const int*, int, int, int);
  void (*refine)(cpra_plan_t, const RefineArgs&);
  void (*fused_step)(cpra_plan_t const*, int, bool, int, double, hipStream_t);
  void (*synth)(cpra_plan_t, int, int, uint64_t);
};

template <int N, typename T, typename AP>
struct Impl {
  using C = cx<T>;
  static void twiddles(cpra_plan_t pl) {
    k_twiddles<N, T><<<(TwLayout<N>::SIZE + 255) / 256, 256, 0, pl->stream>>>(at<C>(pl, pl->L.tw));
  }
  static void prep(cpra_plan_t pl, const float* I, const uint8_t* S, int first, int count) {
    double* psum = at<double>(pl, pl->L.prep_part);
    float* pmax = reinterpret_cast<float*>(psum + (size_t)pl->p.Np * kPrepBlocks);
    k_prep_stats<N><<<dim3(kPrepBlocks, count), 256, 0, pl->stream>>>(I, first, psum, pmax, at<int>(pl, pl->L.flags));
    k_prep_final<T, AP><<<(count + 63) / 64, 64, 0, pl->stream>>>(first, count, psum, pmax, at<double>(pl, pl->L.den),
                                                                  at<T>(pl, pl->L.ampscale));
    k_prep_encode<N, T, AP><<<dim3(N / 8, count), 256, 0, pl->stream>>>(I, S, first, at<AP>(pl, pl->L.A2),
                                                                        at<T>(pl, pl->L.ampscale),
                                                                        at<uint32_t>(pl, pl->L.maskw));
  }
  // initial objects of `count` angles listed at alist (device)
  static void init(cpra_plan_t pl, const int* d_list, int count, int gbuf) {
    using CG = ColGeom<N>;
    using RG = RowGeom<N>;
    dim3 gc(CG::TILES, count), bc(CG::R1 * CG::C);
    if constexpr (CG::S >= 2)
      k_col_pair<N, T, AP, 1, false><<<gc, bc, 0, pl->stream>>>(
          nullptr, at<C>(pl, pl->L.Pmid), at<AP>(pl, pl->L.A2), at<T>(pl, pl->L.ampscale), at<C>(pl, pl->L.tw),
          d_list, nullptr, pl->p.Np, nullptr, CG::TILES, pl->p.seed);
    else
      k_col<N, T, AP, 1, false><<<gc, bc, 0, pl->stream>>>(
          nullptr, at<C>(pl, pl->L.Pmid), at<AP>(pl, pl->L.A2), at<T>(pl, pl->L.ampscale), at<C>(pl, pl->L.tw),
          d_list, nullptr, pl->p.Np, nullptr, CG::TILES, pl->p.seed);
    T* g = at<T>(pl, gbuf ? pl->L.g1 : pl->L.g0);
    dim3 gr(N / RG::RPB, count), br(RG::T * RG::RPB);
    k_row<N, T><<<gr, br, 0, pl->stream>>>(at<C>(pl, pl->L.Pmid), at<C>(pl, pl->L.P), g, g,
                                          at<uint32_t>(pl, pl->L.maskw), at<C>(pl, pl->L.tw), d_list, nullptr,
                                          pl->p.Np, 0, (T)0, pl->p.positivity);
  }
  // one iteration of the listed slots; couple: Eq. 4 on the way in, from buffer cur into the other
  // buffer (Jacobi) or, with inplace, within buffer cur (the neighbours must not be listed)
  // pin / gbuf (when non-NULL / >= 0): column-pass input spectra and the g buffer to run on,
  // instead of P and buffer cur (a K-tap boundary couples into the Pc planes first)
  static void step(cpra_plan_t pl, const int* al, int nact, bool couple, bool inplace, int mode, double beta,
                   double* errpart, const void* pin, int gbuf) {
    using CG = ColGeom<N>;
    using RG = RowGeom<N>;
    dim3 gc(CG::TILES, nact), bc(CG::R1 * CG::C);
    const cpra::Coupling* cp = at<cpra::Coupling>(pl, pl->L.coup);
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (pl->timing) {
      e0 = pl->next_event(); e1 = pl->next_event(); e2 = pl->next_event();
      if (e0) (void)hipEventRecord(e0, pl->stream);
    }
    auto launch = [&](auto kern, double* ep) {
      kern<<<gc, bc, 0, pl->stream>>>(pin ? reinterpret_cast<const C*>(pin) : at<C>(pl, pl->L.P),
                                      at<C>(pl, pl->L.Pmid), at<AP>(pl, pl->L.A2),
                                      at<T>(pl, pl->L.ampscale), at<C>(pl, pl->L.tw), al, cp, pl->p.Np, ep,
                                      CG::TILES, 0);
    };
    if constexpr (CG::S >= 2) {
      if (couple) {
        if (errpart) launch(k_col_pair<N, T, AP, 0, true, true>, errpart);
        else launch(k_col_pair<N, T, AP, 0, false, true>, nullptr);
      } else {
        if (errpart) launch(k_col_pair<N, T, AP, 0, true, false>, errpart);
        else launch(k_col_pair<N, T, AP, 0, false, false>, nullptr);
      }
    } else {
      if (couple) {
        if (errpart) launch(k_col<N, T, AP, 0, true, true>, errpart);
        else launch(k_col<N, T, AP, 0, false, true>, nullptr);
      } else {
        if (errpart) launch(k_col<N, T, AP, 0, true, false>, errpart);
        else launch(k_col<N, T, AP, 0, false, false>, nullptr);
      }
    }
    if (e1) (void)hipEventRecord(e1, pl->stream);
    const int gb = gbuf >= 0 ? gbuf : pl->cur;
    T* gin = at<T>(pl, gb ? pl->L.g1 : pl->L.g0);
    T* gout = (couple && !inplace) ? at<T>(pl, gb ? pl->L.g0 : pl->L.g1) : gin;
    // the row pass with the plan's tile height (results do not depend on it)
    auto row = [&](auto kern, int rpb) {
      kern<<<dim3(N / rpb, nact), dim3(RG::T * rpb), 0, pl->stream>>>(
          at<C>(pl, pl->L.Pmid), at<C>(pl, pl->L.P), gin, gout, at<uint32_t>(pl, pl->L.maskw), at<C>(pl, pl->L.tw), al,
          cp, pl->p.Np, mode, (T)beta, pl->p.positivity);
    };
    constexpr int R0 = RowRows<N, 0>::RPB, R1 = RowRows<N, 1>::RPB;
    if (pl->row_alt) {
      if (couple) row(k_row<N, T, true, R1>, R1);
      else row(k_row<N, T, false, R1>, R1);
    } else {
      if (couple) row(k_row<N, T, true, R0>, R0);
      else row(k_row<N, T, false, R0>, R0);
    }
    if (e2) (void)hipEventRecord(e2, pl->stream);
  }
  // E_F partials of the current iterates of the listed slots (column pass without coupling; its
  // Pmid output is scratch)
  static void colerr(cpra_plan_t pl, const int* al, int nact, double* errpart) {
    using CG = ColGeom<N>;
    dim3 gc(CG::TILES, nact), bc(CG::R1 * CG::C);
    auto kern = [&]() {
      if constexpr (CG::S >= 2) return k_col_pair<N, T, AP, 0, true, false>;
      else return k_col<N, T, AP, 0, true, false>;
    }();
    kern<<<gc, bc, 0, pl->stream>>>(at<C>(pl, pl->L.P), at<C>(pl, pl->L.Pmid), at<AP>(pl, pl->L.A2),
                                    at<T>(pl, pl->L.ampscale), at<C>(pl, pl->L.tw), al, nullptr, pl->p.Np, errpart,
                                    CG::TILES, 0);
  }
  static void moments(cpra_plan_t pl, const int* list, int count, double* out) {
    k_moments<N, T><<<count, 256, 0, pl->stream>>>(at<T>(pl, pl->cur ? pl->L.g1 : pl->L.g0), list, out);
  }
  static void twin(cpra_plan_t pl, const int* slot, const int* shift, int count, double* out) {
    k_twin_dist<N, T><<<count, 256, 0, pl->stream>>>(at<T>(pl, pl->cur ? pl->L.g1 : pl->L.g0), slot, shift, out);
  }
  static void merge_avg(cpra_plan_t pl, int K, const int* keep, const int* inv, const int* shift, void* out) {
    k_merge_avg<N, T><<<dim3(N, pl->p.Np), 256, 0, pl->stream>>>(at<T>(pl, pl->cur ? pl->L.g1 : pl->L.g0),
                                                                 pl->p.Np, K, keep, inv, shift,
                                                                 reinterpret_cast<T*>(out));
  }
  // row spectra P = F_t(g) of the listed angles from the iterate in buffer gbuf
  static void reload(cpra_plan_t pl, const int* d_list, int count, int gbuf) {
    using RG = RowGeom<N>;
    T* g = at<T>(pl, gbuf ? pl->L.g1 : pl->L.g0);
    dim3 gr(N / RG::RPB, count), br(RG::T * RG::RPB);
    k_row<N, T><<<gr, br, 0, pl->stream>>>(nullptr, at<C>(pl, pl->L.P), g, g, at<uint32_t>(pl, pl->L.maskw),
                                          at<C>(pl, pl->L.tw), d_list, nullptr, pl->p.Np, 3, (T)0,
                                          pl->p.positivity);
  }
  // support of the listed slots (one guess: slot = data angle) from their current objects; the
  // blurred planes use the Pmid scratch, the window taps sit at L.swk, partial maxima at errpart
  static void shrinkwrap(cpra_plan_t pl, const int* list, int count, int W, double frac) {
    constexpr int CB = 8;
    T* buf = at<T>(pl, pl->L.Pmid);
    double* pm = at<double>(pl, pl->L.errpart);
    k_blur_rows<N, T><<<dim3(N, count), 256, 0, pl->stream>>>(at<T>(pl, pl->cur ? pl->L.g1 : pl->L.g0), list,
                                                              at<T>(pl, pl->L.swk), W, buf);
    k_blur_cols<N, T, CB><<<dim3(N / CB, count), 256, 0, pl->stream>>>(buf, at<T>(pl, pl->L.swk), W, pm);
    k_shrink_mask<N, T, CB><<<dim3(N, count), 256, 0, pl->stream>>>(buf, list, pm, frac,
                                                                    at<uint32_t>(pl, pl->L.maskw));
  }
  // Eq. 4 with 2K+1 taps for the listed slots: P -> Pc, g[gin_buf] -> g[gout_buf]
  static void couple_taps(cpra_plan_t pl, const int* al, int nact, int gin_buf, int gout_buf) {
    k_couple_taps<N, T><<<dim3(N, nact), 256, 0, pl->stream>>>(
        at<C>(pl, pl->L.P), at<C>(pl, pl->L.Pc), at<T>(pl, gin_buf ? pl->L.g1 : pl->L.g0),
        at<T>(pl, gout_buf ? pl->L.g1 : pl->L.g0), al, at<cpra::Tap>(pl, pl->L.ctab), 2 * pl->K + 1);
  }
  static void refine(cpra_plan_t pl, const RefineArgs& a) {
    constexpr int CB = 8;
    C* tw = at<C>(pl, pl->L.tw);
    T* V = reinterpret_cast<T*>(a.vol);
    C* Q = reinterpret_cast<C*>(a.qh);
    C* Cb = reinterpret_cast<C*>(a.cb);
    const bool bil = pl->p.insertion == CPRA_INSERT_BILINEAR;
    k_ref_gather<N, T><<<dim3(N, N), 256, 0, pl->stream>>>(at<C>(pl, pl->L.P), at<int>(pl, pl->L.csr_ptr),
                                                           at<int>(pl, pl->L.csr_ent),
                                                           bil ? at<T>(pl, pl->L.csr_w) : nullptr,
                                                           at<T>(pl, pl->L.cnt_inv), Q);
    k_ref_support<N><<<dim3(N, N), 256, 0, pl->stream>>>(at<uint32_t>(pl, pl->L.maskw), a.list, a.sc, a.count,
                                                         a.s3);
    const unsigned rows = (unsigned)((size_t)N * N / kRefLines);
    const int rthreads = StepdCfg<N>::R1 * kRefLines;
    k_ref_rows<N, T, true><<<rows, rthreads, 0, pl->stream>>>(Cb, V, a.s3, pl->p.positivity, tw);
    for (int it = 1; it <= a.n_iter; ++it) {
      k_ref_cols<N, T><<<dim3(N / kRefLines, N), rthreads, 0, pl->stream>>>(Cb, Q, tw);
      k_ref_rows<N, T, false><<<rows, rthreads, 0, pl->stream>>>(Cb, V, a.s3, pl->p.positivity, tw);
      if (a.shrink_every > 0 && it % a.shrink_every == 0) {
        // separable blur of V along x, y (planes as slots 0..N-1) and z into Cb, then threshold
        T* buf = reinterpret_cast<T*>(Cb);
        const T* win = reinterpret_cast<const T*>(a.win);
        k_blur_rows<N, T><<<dim3(N, N), 256, 0, pl->stream>>>(V, a.list + a.count, win, a.W, buf);
        k_blur_cols<N, T, CB><<<dim3(N / CB, N), 256, 0, pl->stream>>>(buf, win, a.W, a.pmax);
        k_blur_z<N, T, CB><<<dim3(N / CB, N), 256, 0, pl->stream>>>(buf, win, a.W, a.pmax);
        k_max_reduce<<<1, 256, 0, pl->stream>>>(a.pmax, N * (N / CB));
        k_threshold<T><<<4096, 256, 0, pl->stream>>>(buf, (size_t)N * N * N, a.pmax + N * (N / CB), a.threshold,
                                                     a.s3);
        k_ref_rows<N, T, true><<<rows, rthreads, 0, pl->stream>>>(Cb, V, a.s3, pl->p.positivity, tw);
      }
    }
  }
  // one iteration of `count` plans of this size and precision, one launch per pass for every
  // kFuseMax plans, on stream st: each plan's listed slots (its alist), all coupled at a boundary
  // or none, all in row-pass `mode`.  Same arithmetic per slot as `step`.
  static void fused_step(cpra_plan_t const* pls, int count, bool couple, int mode, double beta, hipStream_t st) {
    using CG = ColGeom<N>;
    using RG = RowGeom<N>;
    for (int b0 = 0; b0 < count; b0 += kFuseMax) {
      const int bn = count - b0 < kFuseMax ? count - b0 : kFuseMax;
      FuseTab<T, AP> ft{};
      ft.count = bn;
      int tot = 0;
      for (int i = 0; i < bn; ++i) {
        cpra_plan_t pl = pls[b0 + i];
        FusePlan<T, AP>& q = ft.p[i];
        ft.start[i] = tot;
        q.P = at<C>(pl, pl->L.P);
        q.Pmid = at<C>(pl, pl->L.Pmid);
        q.A2 = at<AP>(pl, pl->L.A2);
        q.ampscale = at<T>(pl, pl->L.ampscale);
        q.tw = at<C>(pl, pl->L.tw);
        q.alist = at<int>(pl, pl->L.alist);
        q.coup = at<cpra::Coupling>(pl, pl->L.coup);
        q.gin = at<T>(pl, pl->cur ? pl->L.g1 : pl->L.g0);
        q.gout = at<T>(pl, (couple ? pl->cur ^ 1 : pl->cur) ? pl->L.g1 : pl->L.g0);
        q.maskw = at<uint32_t>(pl, pl->L.maskw);
        q.npd = pl->p.Np;
        q.positivity = pl->p.positivity;
        tot += (int)pl->alist_h.size();
      }
      ft.start[bn] = tot;
      if (tot == 0) continue;
      dim3 gc(CG::TILES, tot), bc(CG::R1 * CG::C);
      if constexpr (CG::S >= 2) {
        if (couple) k_colpair_fused<N, T, AP, true><<<gc, bc, 0, st>>>(ft);
        else k_colpair_fused<N, T, AP, false><<<gc, bc, 0, st>>>(ft);
      } else {
        if (couple) k_col_fused<N, T, AP, true><<<gc, bc, 0, st>>>(ft);
        else k_col_fused<N, T, AP, false><<<gc, bc, 0, st>>>(ft);
      }
      constexpr int R0 = RowRows<N, 0>::RPB, R1 = RowRows<N, 1>::RPB;
      const int rpb = pls[b0]->row_alt ? R1 : R0;
      dim3 gr(N / rpb, tot), br(RG::T * rpb);
      if (pls[b0]->row_alt) {
        if (couple) k_row_fused<N, T, AP, true, R1><<<gr, br, 0, st>>>(ft, mode, (T)beta);
        else k_row_fused<N, T, AP, false, R1><<<gr, br, 0, st>>>(ft, mode, (T)beta);
      } else {
        if (couple) k_row_fused<N, T, AP, true, R0><<<gr, br, 0, st>>>(ft, mode, (T)beta);
        else k_row_fused<N, T, AP, false, R0><<<gr, br, 0, st>>>(ft, mode, (T)beta);
      }
    }
  }
  // a synthetic scan of `count` angles from `first` into the plan's staging buffers (autotuning)
  static void synth(cpra_plan_t pl, int first, int count, uint64_t seed) {
    k_synth_scan<N><<<dim3(N, count), 256, 0, pl->stream>>>(at<float>(pl, pl->L.stage_I),
                                                           at<uint8_t>(pl, pl->L.stage_S), first, seed);
  }
  static void assemble(cpra_plan_t pl, void* vol) {
    stepd_run<N, T>(at<C>(pl, pl->L.P), pl->p.Np, at<C>(pl, pl->L.stage_T), at<CellRec>(pl, pl->L.csr_cell),
                    at<CellRec>(pl, pl->L.csr_heavy), pl->n_heavy, at<int>(pl, pl->L.csr_ent),
                    pl->p.insertion == CPRA_INSERT_BILINEAR ? at<T>(pl, pl->L.csr_w) : nullptr,
                    at<T>(pl, pl->L.cnt_inv), at<C>(pl, pl->L.tw), at<C>(pl, pl->L.plane), pl->L.zc,
                    reinterpret_cast<T*>(vol), pl->stream);
  }
};



template <int N, typename T, typename AP> Ops ops_for() {
  return Ops{&Impl<N, T, AP>::twiddles, &Impl<N, T, AP>::prep,    &Impl<N, T, AP>::init,
             &Impl<N, T, AP>::step,     &Impl<N, T, AP>::assemble, &Impl<N, T, AP>::reload,
             &Impl<N, T, AP>::colerr,   &Impl<N, T, AP>::moments,  &Impl<N, T, AP>::twin,
             &Impl<N, T, AP>::merge_avg, &Impl<N, T, AP>::shrinkwrap, &Impl<N, T, AP>::couple_taps,
             &Impl<N, T, AP>::refine, &Impl<N, T, AP>::fused_step, &Impl<N, T, AP>::synth};
}


template <int N> Ops ops_for_size(const cpra_params& p) {
  if (p.real_type == CPRA_REAL_F64) return ops_for<N, double, double2>();
  if (p.amp_type == CPRA_AMP_F16) return ops_for<N, float, __half2>();
  return ops_for<N, float, float2>();
}
extern template Ops ops_for_size<64>(const cpra_params&);
extern template Ops ops_for_size<128>(const cpra_params&);
extern template Ops ops_for_size<192>(const cpra_params&);
extern template Ops ops_for_size<256>(const cpra_params&);
extern template Ops ops_for_size<384>(const cpra_params&);
extern template Ops ops_for_size<512>(const cpra_params&);
extern template Ops ops_for_size<1024>(const cpra_params&);

}  // namespace cpra_impl
