// Segmented launches of a round (see round.h).
#include <string.h>

#include "round.h"

namespace scvt {

bool Round::empty() const { return out.empty(); }

void Round::clear() {
  for (auto& v : push_ext) v.clear();
  fin_chain.clear();
  fin_back.clear();
  fin_fwd.clear();
  fin_gq.clear();
  for (auto& v : q0) v.clear();
  for (auto& v : dir) v.clear();
  norm.clear();
  grid.clear();
  cells.clear();
  cells_all.clear();
  quad.clear();
  reduce.clear();
  fin.clear();
  out.clear();
}

// one block per problem: its scalars into the round's staging
__global__ void k_gather(Many<GatherArgs> p) {
  if (p.idle()) return;
  const GatherArgs& a = p.args();
  for (int k = threadIdx.x; k < a.count; k += blockDim.x) a.dst[k] = a.src[k];
}

hipError_t launch_gather_many(const Seg<GatherArgs>& g, hipStream_t s) {
  k_gather<<<dim3(g.maxnb, g.nseg), 64, 0, s>>>(Many<GatherArgs>{g.tab, g.nb});
  return hipGetLastError();
}

namespace {

// bump layout of the round's tables in the staging buffers
struct Stage {
  RoundBuffers& b;
  size_t used = 0;
  bool overflow = false;
  explicit Stage(RoundBuffers& bb) : b(bb) {}
  template <class T>
  const T* put(const T* data, size_t count) {
    const size_t at = (used + 255) / 256 * 256, bytes = count * sizeof(T);
    if (at + bytes > b.bytes) {
      overflow = true;
      return nullptr;
    }
    memcpy((char*)b.host + at, data, bytes);
    used = at + bytes;
    return reinterpret_cast<const T*>((const char*)b.dev + at);
  }
  // a problem list's table and per-problem grid sizes
  template <class T, class F>
  Seg<T> seg(const std::vector<T>& v, F grid_of) {
    Seg<T> g{nullptr, nullptr, (int)v.size(), 0};
    if (v.empty()) return g;
    std::vector<int32_t> nb(v.size());
    for (size_t k = 0; k < v.size(); k++) {
      nb[k] = grid_of(v[k]);
      if (nb[k] > g.maxnb) g.maxnb = nb[k];
    }
    g.tab = put(v.data(), v.size());
    g.nb = put(nb.data(), nb.size());
    return g;
  }
};

}  // namespace

hipError_t round_run(Round& r, RoundBuffers& b, hipStream_t s) {
  Stage st(b);
  auto hist = [](const auto& a) { return hist_grid(a.n3); };
  auto one = [](const auto&) { return 1; };
  Seg<PushExtArgs> pe[2] = {st.seg(r.push_ext[0], hist), st.seg(r.push_ext[1], hist)};
  Seg<FinChain> fc = st.seg(r.fin_chain, one);
  Seg<HistFinArgs> fb = st.seg(r.fin_back, one), ff = st.seg(r.fin_fwd, one),
                   fg = st.seg(r.fin_gq, one);
  Seg<HistPassArgs> q0[2] = {st.seg(r.q0[0], hist), st.seg(r.q0[1], hist)};
  Seg<HistPassArgs> dr[2] = {st.seg(r.dir[0], hist), st.seg(r.dir[1], hist)};
  Seg<NormArgs> nm = st.seg(r.norm, [](const NormArgs& a) { return normalize_grid(a.n); });
  Seg<GridBuildArgs> gb = st.seg(r.grid, [](const GridBuildArgs& a) { return bucket_grid(a.n); });
  std::vector<ScanArgs> scans;
  for (const auto& a : r.grid) scans.push_back(grid_scan_args(a.gb));
  Seg<ScanArgs> sc_tiles = st.seg(scans, [](const ScanArgs& a) { return (int)a.ntiles; });
  Seg<ScanArgs> sc_one = sc_tiles;
  if (!scans.empty()) {
    std::vector<int32_t> ones(scans.size(), 1);
    sc_one.nb = st.put(ones.data(), ones.size());
    sc_one.maxnb = 1;
  }
  // the cell kernels: one table, a grid size per kernel and problem
  std::vector<CellArgs> cl = r.cells;
  cl.insert(cl.end(), r.cells_all.begin(), r.cells_all.end());
  const size_t nmain = r.cells.size();
  std::vector<int32_t> g_main(cl.size()), g_t0(cl.size()), g_t1(cl.size()), g_all(cl.size()),
      g_fb(cl.size());
  int m_main = 0, m_t0 = 0, m_t1 = 0, m_all = 0, m_fb = 0;
  for (size_t k = 0; k < cl.size(); k++) {
    const bool main = k < nmain;
    const int64_t n = cl[k].n;
    g_main[k] = main ? cells_main_grid(n) : 0;
    g_t0[k] = main ? cells_tier_grid(n, 0) : 0;
    g_t1[k] = main ? cells_tier_grid(n, 1) : 0;
    g_all[k] = main ? 0 : fb_all_grid(n);
    g_fb[k] = cells_fallback_grid(n, main ? 0 : 1);
    m_main = g_main[k] > m_main ? g_main[k] : m_main;
    m_t0 = g_t0[k] > m_t0 ? g_t0[k] : m_t0;
    m_t1 = g_t1[k] > m_t1 ? g_t1[k] : m_t1;
    m_all = g_all[k] > m_all ? g_all[k] : m_all;
    m_fb = g_fb[k] > m_fb ? g_fb[k] : m_fb;
  }
  const CellArgs* cl_tab = cl.empty() ? nullptr : st.put(cl.data(), cl.size());
  const int32_t* cl_nb[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!cl.empty()) {
    cl_nb[0] = st.put(g_main.data(), cl.size());
    cl_nb[1] = st.put(g_t0.data(), cl.size());
    cl_nb[2] = st.put(g_t1.data(), cl.size());
    cl_nb[3] = st.put(g_all.data(), cl.size());
    cl_nb[4] = st.put(g_fb.data(), cl.size());
  }
  std::vector<std::pair<std::pair<int, int>, Seg<CellArgs>>> qd;
  for (const auto& kv : r.quad)
    qd.push_back({kv.first, st.seg(kv.second, [](const CellArgs& a) { return quad_grid(a.n); })});
  Seg<EvalRedArgs> rd = st.seg(r.reduce, [](const EvalRedArgs& a) { return reduce_grid(a.n); });
  Seg<FinalizeArgs> fn = st.seg(r.fin, one);
  // scalars: each problem's values into one staging array
  std::vector<GatherArgs> ga;
  int nscal = 0;
  for (const auto& o : r.out) {
    ga.push_back(GatherArgs{o.src, b.dscal + nscal, o.count});
    nscal += o.count;
  }
  if (nscal > b.max_scal) return hipErrorInvalidValue;
  Seg<GatherArgs> gs = st.seg(ga, one);
  if (st.overflow) return hipErrorInvalidValue;

  hipError_t e = hipSuccess;
#define RCK(x)              \
  do {                      \
    e = (x);                \
    if (e != hipSuccess) return e; \
  } while (0)
  if (st.used) RCK(hipMemcpyAsync(b.dev, b.host, st.used, hipMemcpyHostToDevice, s));
  for (int w = 0; w < 2; w++)
    if (pe[w].nseg) RCK(launch_push_ext_many(pe[w], w + 1, s));
  if (fc.nseg) RCK(launch_fin_chain_many(fc, s));
  if (fb.nseg) RCK(launch_hist_fin_many(fb, s));
  for (int w = 0; w < 2; w++)
    if (q0[w].nseg) RCK(launch_hist_q0_many(q0[w], w + 1, s));
  if (ff.nseg) RCK(launch_hist_fin_many(ff, s));
  for (int w = 0; w < 2; w++)
    if (dr[w].nseg) RCK(launch_hist_dir_many(dr[w], w + 1, s));
  if (fg.nseg) RCK(launch_hist_fin_many(fg, s));
  if (nm.nseg) RCK(launch_normalize_trial_many(nm, s));
  if (gb.nseg) RCK(launch_grid_build_many(gb, sc_tiles, sc_one, s));
  if (!cl.empty())
    RCK(launch_cells_many(cl_tab, cl_nb[0], m_main, cl_nb[1], m_t0, cl_nb[2], m_t1, cl_nb[3], m_all,
                          cl_nb[4], m_fb, (int)cl.size(), s));
  for (const auto& q : qd) RCK(launch_quad_many(q.second, q.first.first, q.first.second, s));
  if (rd.nseg) RCK(launch_eval_reduce_many(rd, s));
  if (fn.nseg) RCK(launch_finalize_many(fn, s));
  if (gs.nseg) {
    RCK(launch_gather_many(gs, s));
    RCK(hipMemcpyAsync(b.hscal, b.dscal, nscal * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  RCK(hipStreamSynchronize(s));
#undef RCK
  int at = 0;
  for (const auto& o : r.out) {
    memcpy(o.host, b.hscal + at, o.count * sizeof(double));
    at += o.count;
  }
  return hipSuccess;
}

}  // namespace scvt
