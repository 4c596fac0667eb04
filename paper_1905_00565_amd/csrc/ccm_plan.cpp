// ccm_plan.cpp -- validation of a call and layout of its realizations,
// work items and device pools (the planner of libccm).
#include <numeric>
#include <unordered_map>

#include "ccm_host.h"

namespace ccmh {

OrderKey embedding_order(int32_t E, int32_t tau) {
  if (E == 1) return {1, {0, 0, 0, 0}};
#ifndef CCM_KD_MIN_E
#define CCM_KD_MIN_E 3
#endif
  if (E < CCM_KD_MIN_E) return {2, {0, tau, 0, 0}};
  // sorted first on the newest coordinate, which puts exactly the embedded
  // points (i < n_e) first; the k-d levels then reorder them
  return {1, {(E - 1) * tau, 0, 0, 0}, E};
}

// Leaves of about this many points end the k-d refinement.
#ifndef CCM_KD_LEAF
#define CCM_KD_LEAF 48
#endif
constexpr int64_t kKdLeaf = CCM_KD_LEAF;
constexpr int kKdMaxLevels = 12;

void attach_kd(Plan& p, int64_t key_off, int32_t E, int64_t emb_off, int64_t ne) {
  OrderJob& o = p.orders[(size_t)(key_off / p.spec.N)];
  if (o.kd_E == 0) return;
  o.kd_emb_off = emb_off;
  o.kd_n_e = ne;
  int lv = 1;
  while (lv < kKdMaxLevels && (ne >> lv) > kKdLeaf) ++lv;
  o.kd_levels = lv;
  p.kd_levels = std::max(p.kd_levels, lv);
  (void)E;
}

void size_order_sort(Plan& p) {
  HIPCHK(sort_series(nullptr, p.sort_temp, nullptr, nullptr, nullptr, nullptr, p.spec.N,
                     p.n_sets, nullptr, nullptr));
}

OrderKey shared_order(int32_t Emax, int32_t tau) {
  if (Emax == 1) return {1, {0, 0, 0, 0}};
  if (Emax < 6) return {2, {(Emax - 2) * tau, (Emax - 1) * tau, 0, 0}};
  return {4, {(Emax - 1) * tau, (Emax - 2) * tau, (Emax - 3) * tau, (Emax - 4) * tau}};
}

int64_t order_set(Plan& p, int series, const OrderKey& key) {
  const int64_t N = p.spec.N;
  for (size_t k = 0; k < p.orders.size(); ++k) {
    const OrderJob& o = p.orders[k];
    if (o.src_off == series * N && o.dims == key.dims && o.kd_E == key.kd_E &&
        std::equal(key.lag, key.lag + 4, o.lag))
      return o.key_off;
  }
  const int64_t off = (int64_t)p.orders.size() * N;
  OrderJob o{};
  o.src_off = series * N;
  o.key_off = off;
  o.n = N;
  o.dims = key.dims;
  for (int d = 0; d < 4; ++d) o.lag[d] = key.lag[d];
  o.kd_E = key.kd_E;
  p.orders.push_back(o);
  p.n_sets = (int32_t)p.orders.size();
  p.n_ord = p.n_sets * N;
  if (p.n_ord > (int64_t)INT32_MAX) fail(CCM_E_INVAL, "too many time points to order");
  p.seg_off.clear();
  for (int k = 0; k <= p.n_sets; ++k) p.seg_off.push_back((int32_t)(k * N));
  return off;
}

// A realization walks a table when the flag asks for it, its embedding fits
// the walk's LDS bitmask, the expected walk to E+1 acceptable library members
// ((E+1+excluded) n_e / l_eff row entries) is at most a quarter of a
// truncated row (a wavefront whose walk runs short scans instead, which must
// stay rare), and the walk (about 8 instructions per entry) is cheaper than
// the scan (2E per pair).
bool use_table(const Plan& p, int E, int64_t ne, int64_t le) {
  if (!(p.spec.flags & CCM_FLAG_TABLE) || ne > kTableMaxNe) return false;
  const double excl =
      p.mode == kExclSelf ? 1.0 : (p.mode == kWindow ? 2.0 * p.window + 1.0 : 0.0);
  const double walk = (E + 1 + excl) * (double)ne / (double)le;
  const int64_t w = std::min<int64_t>(kTableWidth, ne);
  if (w < ne && walk > (double)w / 4.0) return false;
  return 8.0 * walk < 2.0 * E * (double)le;
}

int64_t table_for(Plan& p, int64_t emb_off, int64_t ne, int E) {
  for (const TableJob& t : p.tables)
    if (t.emb_off == emb_off) return t.out_off;
  const int32_t w = (int32_t)std::min<int64_t>(kTableWidth, ne);
  TableJob t{};
  t.emb_off = emb_off;
  t.out_off = p.n_table;
  t.n_e = (int32_t)ne;
  t.E = E;
  t.w = w;
  if (p.te_count[E] == 0) p.te_first[E] = (int)p.tables.size();
  p.te_count[E] += 1;
  p.te_max_ne[E] = std::max(p.te_max_ne[E], (int)ne);
  p.tables.push_back(t);
  p.n_table += ne * table_row_stride(w);
  return t.out_off;
}

uint64_t default_wave_limit(uint64_t total) {
  return std::max<uint64_t>(1ull << 30, std::min<uint64_t>(8ull << 30, total / 8));
}

// Pool bytes of one realization in its wave: its gathered library (binary32
// coordinates and int32 indices), and, once per wave, its library draw (a
// nested shuffle also keeps its n_e positions).
static uint64_t draw_bytes(const Plan& p, int64_t sj) {
  if (!p.nested.empty()) return ((uint64_t)p.nested[sj].n_out + (uint64_t)p.nested[sj].n_e) * 4;
  return (uint64_t)p.sample[sj].l_eff * 4;
}
static uint64_t points_bytes(const Realization& R) {
  return (uint64_t)R.l_eff * (uint64_t)(R.E + 1) * 4;
}

// Group the realizations into waves whose pools fit spec.wave_limit (0: one
// wave): all realizations of one E together when they fit, consecutive E
// merged while they fit, an E too large for one wave split into several.
// Then lay out each wave's draws and gathered libraries from offset 0 of
// the shared pools (a draw used by realizations of two waves is drawn in
// both) and rebase the realizations and jobs that refer to them.
static void split_waves(Plan& p) {
  const uint64_t limit = p.spec.wave_limit;
  const bool nested = !p.nested.empty();
  const size_t n = p.rz.size();
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return p.rz[a].E < p.rz[b].E; });

  std::vector<std::vector<int32_t>> waves;
  std::vector<int32_t> cur;
  std::unordered_map<int64_t, int> cur_draws;
  uint64_t cur_b = 0;
  auto close_wave = [&] {
    if (!cur.empty()) waves.push_back(std::move(cur));
    cur.clear();
    cur_draws.clear();
    cur_b = 0;
  };
  auto add = [&](int32_t r) {
    cur.push_back(r);
    cur_b += points_bytes(p.rz[r]);
    if (cur_draws.emplace(p.rz_sample[r], 1).second) cur_b += draw_bytes(p, p.rz_sample[r]);
  };
  for (size_t g0 = 0; g0 < n;) {
    size_t g1 = g0;
    while (g1 < n && p.rz[order[g1]].E == p.rz[order[g0]].E) ++g1;
    // bytes of the whole E group (its draws counted once each)
    uint64_t gb = 0;
    {
      std::unordered_map<int64_t, int> d;
      for (size_t k = g0; k < g1; ++k) {
        gb += points_bytes(p.rz[order[k]]);
        if (d.emplace(p.rz_sample[order[k]], 1).second) gb += draw_bytes(p, p.rz_sample[order[k]]);
      }
    }
    if (limit == 0 || cur_b + gb <= limit) {
      for (size_t k = g0; k < g1; ++k) add(order[k]);
    } else if (gb <= limit) {
      close_wave();
      for (size_t k = g0; k < g1; ++k) add(order[k]);
    } else {
      close_wave();
      for (size_t k = g0; k < g1; ++k) {
        const int32_t r = order[k];
        uint64_t b = points_bytes(p.rz[r]);
        if (!cur_draws.count(p.rz_sample[r])) b += draw_bytes(p, p.rz_sample[r]);
        if (!cur.empty() && cur_b + b > limit) close_wave();
        add(r);
      }
    }
    g0 = g1;
  }
  close_wave();

  std::vector<SampleJob> sample;
  std::vector<NestedJob> shuffles;
  std::vector<GatherJob> gather;
  int64_t max_lib = 0, max_pts = 0, max_pj = 0, max_scr = 0;
  p.waves.clear();
  p.wave_rz.clear();
  p.wave_rz_first.clear();
  for (const auto& wr : waves) {
    Wave w;
    w.sample_first = nested ? (int64_t)shuffles.size() : (int64_t)sample.size();
    w.gather_first = (int64_t)gather.size();
    p.wave_rz_first.push_back((int64_t)p.wave_rz.size());
    std::unordered_map<int64_t, int64_t> remap;   // draw: old index -> new index
    int64_t lib = 0, pts = 0, pj = 0, scr = 0;
    for (int32_t r : wr) {
      p.wave_rz.push_back(r);
      const int64_t sj = p.rz_sample[r];
      int64_t old_out = 0, new_out = 0;
      auto it = remap.find(sj);
      if (nested) {
        old_out = p.nested[sj].out_off;
        if (it == remap.end()) {
          NestedJob j = p.nested[sj];
          j.out_off = lib;
          j.scratch_off = scr;
          lib += j.n_out;
          scr += j.n_e;
          it = remap.emplace(sj, (int64_t)shuffles.size()).first;
          shuffles.push_back(j);
        }
        new_out = shuffles[it->second].out_off;
      } else {
        old_out = p.sample[sj].out_off;
        if (it == remap.end()) {
          SampleJob j = p.sample[sj];
          j.out_off = lib;
          lib += j.l_eff;
          it = remap.emplace(sj, (int64_t)sample.size()).first;
          sample.push_back(j);
        }
        new_out = sample[it->second].out_off;
      }
      Realization& R = p.rz[r];
      const int64_t ng = nested ? R.n_seg : 1;
      const int64_t g0 = p.rz_gather[r];
      p.rz_gather[r] = (int64_t)gather.size();
      for (int64_t g = g0; g < g0 + ng; ++g) {
        GatherJob G = p.gather[g];
        G.lib_off = new_out + (G.lib_off - old_out);
        G.pts_off = pts + (G.pts_off - R.pts_off);
        G.pj_off = pj + (G.pj_off - R.pj_off);
        if (G.sorted) w.max_sorted_n_e = std::max(w.max_sorted_n_e, G.n_e);
        gather.push_back(G);
      }
      p.rz_sample[r] = it->second;
      R.pts_off = pts;
      R.pj_off = pj;
      pts += (int64_t)R.l_eff * R.E;
      pj += R.l_eff;
    }
    w.sample_count = (nested ? (int64_t)shuffles.size() : (int64_t)sample.size()) - w.sample_first;
    w.gather_count = (int64_t)gather.size() - w.gather_first;
    w.pool_bytes = (uint64_t)(lib + pj + scr) * 4 + (uint64_t)pts * 4;
    p.waves.push_back(w);
    max_lib = std::max(max_lib, lib);
    max_pts = std::max(max_pts, pts);
    max_pj = std::max(max_pj, pj);
    max_scr = std::max(max_scr, scr);
  }
  p.wave_rz_first.push_back((int64_t)p.wave_rz.size());
  if (nested)
    p.nested = std::move(shuffles);
  else
    p.sample = std::move(sample);
  p.gather = std::move(gather);
  p.n_lib = max_lib;
  p.n_pts = max_pts;
  p.n_pj = max_pj;
  if (nested) p.n_scratch = max_scr;
}

// Waves, then the work items of each wave grouped by E (one launch each),
// the costliest first within a group: a scan costs n_query * l_eff pairs, a
// table walk about n_query * (E+1) n_e / l_eff row entries.
static void order_items(Plan& p) {
  split_waves(p);
  auto cost = [&](const Realization& R) {
    return R.table_off >= 0 ? (double)R.n_query * (R.E + 1) * R.n_e / R.l_eff / 8.0
                            : (double)R.n_query * R.l_eff;
  };
  for (size_t w = 0; w < p.waves.size(); ++w) {
    std::vector<int32_t> order(p.wave_rz.begin() + p.wave_rz_first[w],
                               p.wave_rz.begin() + p.wave_rz_first[w + 1]);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      if (p.rz[a].E != p.rz[b].E) return p.rz[a].E < p.rz[b].E;
      return cost(p.rz[a]) > cost(p.rz[b]);
    });
    p.waves[w].launch_first = (int32_t)p.launches.size();
    for (int32_t idx : order) {
      const Realization& R = p.rz[idx];
      if (p.launches.size() == (size_t)p.waves[w].launch_first || p.launches.back().E != R.E)
        p.launches.push_back({R.E, (int32_t)p.items.size(), 0});
      for (int t = 0; t < R.n_tiles; ++t) p.items.push_back({idx, t});
      p.launches.back().count += R.n_tiles;
      if (p.items.size() > (size_t)INT32_MAX) fail(CCM_E_INVAL, "too many work items");
    }
    p.waves[w].launch_count = (int32_t)p.launches.size() - p.waves[w].launch_first;
  }
}

// Nested libraries: per (E, tau) the distinct library sizes, sorted, split
// one ordering per r into segments; per (r, direction) one chain whose
// segments are gathered separately (each in visiting order, with its own
// scan starts) and scanned in order, one snapshot per size.
static Plan make_plan_nested(const Spec& s) {
  if (s.query_set != 0) fail(CCM_E_INVAL, "nested libraries predict every embedded point");
  if (s.flags & (CCM_FLAG_TABLE | CCM_FLAG_PLAIN | CCM_FLAG_SHARED_E))
    fail(CCM_E_INVAL,
         "nested libraries do not combine with the table, plain or E-sweep-sharing forms");
  Plan p;
  p.spec = s;
  p.mode = excl_mode(s.excl);
  p.window = s.excl > 0 ? s.excl : 0;
  const int nE = (int)s.E.size(), nT = (int)s.tau.size(), nL = (int)s.L.size();
  const int64_t N = s.N;
  p.n64 = 2 * N;
  p.n32 = 2 * N;
  p.ingest.push_back({0, 0, 2 * N});
  const int64_t sorted_limit = gather_max_sorted_n_e();
  p.n_out = 2LL * nE * nT * nL * s.r;
  p.L_eff.assign((size_t)nE * nT * nL, 0);
  for (int ie = 0; ie < nE; ++ie) {
    const int32_t E = s.E[ie];
    const int Q = crossmap_queries_per_lane(E);
    const int64_t qt = (int64_t)kBlock * Q;
    for (int it = 0; it < nT; ++it) {
      const int32_t tau = s.tau[it];
      const int64_t ne = N - (int64_t)(E - 1) * tau;
      std::vector<int64_t> sizes;
      for (int il = 0; il < nL; ++il) {
        const int64_t le = std::min(s.L[il], ne);
        p.L_eff[((size_t)ie * nT + it) * nL + il] = le;
        sizes.push_back(le);
      }
      std::sort(sizes.begin(), sizes.end());
      sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
      const int n_seg = (int)sizes.size();
      const int64_t lmax = sizes.back();
      const int64_t seg_off = (int64_t)p.segs.size();
      p.segs.push_back(0);
      for (int64_t z : sizes) p.segs.push_back((int32_t)z);
      int64_t emb_off[2], qord_off[2], ord_off[2];
      for (int sr = 0; sr < 2; ++sr) {
        emb_off[sr] = p.n_emb;
        qord_off[sr] = p.n_qord;
        ord_off[sr] = order_set(p, sr, embedding_order(E, tau));
        p.embed.push_back({sr * N, p.n_emb, ord_off[sr], p.n_qord, ne, N, E, tau});
        attach_kd(p, ord_off[sr], E, emb_off[sr], ne);
        p.n_emb += ne * E;
        p.n_qord += ne;
        p.max_embed = std::max(p.max_embed, ne * E);
      }
      const int32_t sorted = ne <= sorted_limit ? 1 : 0;
      if (sorted) p.max_sorted_n_e = std::max(p.max_sorted_n_e, ne);
      for (int ri = 0; ri < s.r; ++ri) {
        NestedJob nj{};
        nj.seed = s.seed;
        nj.n_e = ne;
        nj.n_out = lmax;
        nj.out_off = p.n_lib;
        nj.scratch_off = p.n_scratch;
        nj.E = E;
        nj.tau = tau;
        nj.r_index = ri;
        p.nested.push_back(nj);
        p.n_lib += lmax;
        p.n_scratch += ne;
        for (int dir = 0; dir < 2; ++dir) {
          const int lib_s = dir == 0 ? 1 : 0;
          const int tgt_s = dir == 0 ? 0 : 1;
          Realization R{};
          R.emb_off = emb_off[lib_s];
          R.pts_off = p.n_pts;
          R.pj_off = p.n_pj;
          R.qord_off = qord_off[lib_s];
          R.tgt_off = tgt_s * N;
          R.E = E;
          R.tau = tau;
          R.n_e = (int32_t)ne;
          R.l_eff = (int32_t)lmax;
          R.n_query = (int32_t)ne;
          R.n_tiles = (int32_t)((ne + qt - 1) / qt);
          R.slot_base = p.n_slots;
          R.out_index = -1;
          R.table_off = -1;
          R.n_seg = n_seg;
          R.seg_off = seg_off;
          p.rz_sample.push_back((int64_t)p.nested.size() - 1);
          p.rz_gather.push_back((int64_t)p.gather.size());
          for (int k = 0; k < n_seg; ++k) {
            const int64_t b0 = p.segs[seg_off + k], b1 = p.segs[seg_off + k + 1];
            GatherJob gj{};
            gj.emb_off = R.emb_off;
            gj.lib_off = nj.out_off + b0;
            gj.order_off = ord_off[lib_s];
            gj.pts_off = R.pts_off + b0 * E;
            gj.pj_off = R.pj_off + b0;
            gj.start_off = (R.slot_base + (int64_t)k * R.n_tiles) * kWaves;
            gj.l_eff = b1 - b0;
            gj.n_e = ne;
            gj.n_series = N;
            gj.E = E;
            gj.tau = tau;
            gj.qt = (int32_t)qt;
            gj.query_set = 0;
            gj.sorted = sorted;
            p.gather.push_back(gj);
          }
          for (int il = 0; il < nL; ++il) {
            const int64_t le = p.L_eff[((size_t)ie * nT + it) * nL + il];
            const int k = (int)(std::lower_bound(sizes.begin(), sizes.end(), le) - sizes.begin());
            Realization F{};
            F.slot_base = R.slot_base + (int64_t)k * R.n_tiles;
            F.n_tiles = R.n_tiles;
            F.out_index = ((((int64_t)dir * nE + ie) * nT + it) * nL + il) * s.r + ri;
            p.rz_fin.push_back(F);
            p.preds += (double)ne;
          }
          p.n_pts += lmax * E;
          p.n_pj += lmax;
          p.n_slots += (int64_t)R.n_tiles * n_seg;
          p.rz.push_back(R);
          double pairs = (double)ne * (double)lmax;
          if (p.mode == kExclSelf) pairs -= (double)lmax;
          p.pairs += pairs;
          p.flops += pairs * (3.0 * E - 1.0);
        }
      }
    }
  }
  p.n_rho = (int64_t)p.rz_fin.size();
  if (p.rz.size() > (size_t)INT32_MAX) fail(CCM_E_INVAL, "too many realizations");
  order_items(p);
  size_order_sort(p);
  p.device_bytes = p.n64 * 8 + p.n32 * 4 + p.n_emb * 4 + p.n_lib * 4 + p.n_pts * 4 +
                   p.n_pj * 4 + p.n_qord * 4 + p.n_slots * 4 * kWaves + p.sort_temp +
                   (size_t)p.n_ord * 16 + p.n_scratch * 4 + p.segs.size() * 4 +
                   p.n_slots * sizeof(Moments) + p.n_out * 8 +
                   (p.rz.size() + p.rz_fin.size()) * sizeof(Realization) +
                   p.items.size() * sizeof(Item) + p.nested.size() * sizeof(NestedJob) +
                   p.gather.size() * sizeof(GatherJob);
  return p;
}

// E-sweep sharing: per tau, the embedding of E_max (the largest E asked for)
// over N_c points, one library per (L, r) drawn over them, and one
// realization per (L, r, direction) whose scan keeps a running list for
// every E <= E_max (moments slots: E_max per tile, E's at slot_base +
// (E-1) n_tiles); rz_fin holds one record per requested (E, L, r, direction).
static Plan make_plan_shared(const Spec& s) {
  if (s.query_set != 0) fail(CCM_E_INVAL, "E-sweep sharing predicts every embedded point");
  if (s.flags & (CCM_FLAG_TABLE | CCM_FLAG_PLAIN | CCM_FLAG_NESTED))
    fail(CCM_E_INVAL, "E-sweep sharing does not combine with the table, nested or plain forms");
  Plan p;
  p.spec = s;
  p.mode = excl_mode(s.excl);
  p.window = s.excl > 0 ? s.excl : 0;
  const int nE = (int)s.E.size(), nT = (int)s.tau.size(), nL = (int)s.L.size();
  const int64_t N = s.N;
  const int32_t Emax = *std::max_element(s.E.begin(), s.E.end());
  p.shared_emax = Emax;
  p.n64 = 2 * N;
  p.n32 = 2 * N;
  p.ingest.push_back({0, 0, 2 * N});
  const int64_t sorted_limit = gather_max_sorted_n_e();
  p.n_out = 2LL * nE * nT * nL * s.r;
  p.L_eff.assign((size_t)nE * nT * nL, 0);
  const int64_t qt = (int64_t)kBlock * shared_queries_per_lane(Emax);
  for (int it = 0; it < nT; ++it) {
    const int32_t tau = s.tau[it];
    const int64_t nc = N - (int64_t)(Emax - 1) * tau;
    int64_t emb_off[2], qord_off[2], ord_off[2];
    for (int sr = 0; sr < 2; ++sr) {
      emb_off[sr] = p.n_emb;
      qord_off[sr] = p.n_qord;
      ord_off[sr] = order_set(p, sr, shared_order(Emax, tau));
      p.embed.push_back({sr * N, p.n_emb, ord_off[sr], p.n_qord, nc, N, Emax, tau});
      p.n_emb += nc * Emax;
      p.n_qord += nc;
      p.max_embed = std::max(p.max_embed, nc * Emax);
    }
    const int32_t sorted = nc <= sorted_limit ? 1 : 0;
    if (sorted) p.max_sorted_n_e = std::max(p.max_sorted_n_e, nc);
    for (int il = 0; il < nL; ++il) {
      const int64_t le = std::min(s.L[il], nc);
      for (int ie = 0; ie < nE; ++ie) p.L_eff[((size_t)ie * nT + it) * nL + il] = le;
      for (int ri = 0; ri < s.r; ++ri) {
        const int64_t lib_off = p.n_lib;
        p.sample.push_back({s.seed, nc, le, lib_off, 0, tau, ri, 0});
        p.n_lib += le;
        for (int dir = 0; dir < 2; ++dir) {
          const int lib_s = dir == 0 ? 1 : 0;
          const int tgt_s = dir == 0 ? 0 : 1;
          Realization R{};
          R.emb_off = emb_off[lib_s];
          R.pts_off = p.n_pts;
          R.pj_off = p.n_pj;
          R.qord_off = qord_off[lib_s];
          R.tgt_off = tgt_s * N;
          R.E = Emax;
          R.tau = tau;
          R.n_e = (int32_t)nc;
          R.l_eff = (int32_t)le;
          R.n_query = (int32_t)nc;
          R.n_tiles = (int32_t)((nc + qt - 1) / qt);
          R.slot_base = p.n_slots;
          R.out_index = -1;
          R.table_off = -1;
          GatherJob gj{};
          gj.emb_off = R.emb_off;
          gj.lib_off = lib_off;
          gj.order_off = ord_off[lib_s];
          gj.pts_off = R.pts_off;
          gj.pj_off = R.pj_off;
          gj.start_off = R.slot_base * kWaves;
          gj.l_eff = le;
          gj.n_e = nc;
          gj.n_series = N;
          gj.E = Emax;
          gj.tau = tau;
          gj.qt = (int32_t)qt;
          gj.query_set = 0;
          gj.sorted = sorted;
          p.gather.push_back(gj);
          for (int ie = 0; ie < nE; ++ie) {
            Realization F{};
            F.slot_base = R.slot_base + (int64_t)(s.E[ie] - 1) * R.n_tiles;
            F.n_tiles = R.n_tiles;
            F.out_index = ((((int64_t)dir * nE + ie) * nT + it) * nL + il) * s.r + ri;
            p.rz_fin.push_back(F);
            p.preds += (double)nc;
          }
          p.n_pts += le * Emax;
          p.n_pj += le;
          p.n_slots += (int64_t)R.n_tiles * Emax;
          p.rz.push_back(R);
          p.rz_sample.push_back((int64_t)p.sample.size() - 1);
          p.rz_gather.push_back((int64_t)p.gather.size() - 1);
          // each pair's E_max-coordinate distance is computed once
          double pairs = (double)nc * (double)le;
          if (p.mode == kExclSelf) pairs -= (double)le;
          p.pairs += pairs;
          p.flops += pairs * (3.0 * Emax - 1.0);
        }
      }
    }
  }
  p.n_rho = (int64_t)p.rz_fin.size();
  if (p.rz.size() > (size_t)INT32_MAX) fail(CCM_E_INVAL, "too many realizations");
  order_items(p);
  size_order_sort(p);
  p.device_bytes = p.n64 * 8 + p.n32 * 4 + p.n_emb * 4 + p.n_lib * 4 + p.n_pts * 4 +
                   p.n_pj * 4 + p.n_qord * 4 + p.n_slots * 4 * kWaves + p.sort_temp +
                   (size_t)p.n_ord * 16 + p.n_slots * sizeof(Moments) + p.n_out * 8 +
                   (p.rz.size() + p.rz_fin.size()) * sizeof(Realization) +
                   p.items.size() * sizeof(Item) + p.sample.size() * sizeof(SampleJob) +
                   p.gather.size() * sizeof(GatherJob);
  return p;
}

// Validate a sweep and lay out every realization of it.
Plan make_plan(const Spec& s) {
  if (s.N < 2) fail(CCM_E_INVAL, "N must be >= 2");
  if (s.E.empty() || s.tau.empty() || s.L.empty()) fail(CCM_E_INVAL, "empty E, tau or L list");
  if (s.r < 1) fail(CCM_E_INVAL, "r must be >= 1");
  if (s.query_set != 0 && s.query_set != 1) fail(CCM_E_INVAL, "query_set must be 0 or 1");
  if (s.N > (int64_t)INT32_MAX / 2) fail(CCM_E_INVAL, "N too large");
  for (int32_t e : s.E)
    if (e < 1 || e > kMaxE) fail(CCM_E_INVAL, "E must be in [1, 10]");
  for (int32_t t : s.tau)
    if (t < 1) fail(CCM_E_INVAL, "tau must be >= 1");
  for (int32_t e : s.E)
    for (int32_t t : s.tau) {
      const int64_t ne = s.N - (int64_t)(e - 1) * t;
      if (ne < e + 2) fail(CCM_E_INVAL, "N_e = N - (E-1) tau must be >= E + 2");
      for (int64_t l : s.L) {
        if (l < e + 2) fail(CCM_E_INVAL, "every L must be >= E + 2");
        if (std::min(l, ne) < min_library(e, s.excl))
          fail(CCM_E_INVAL, "library too small for the exclusion window");
      }
    }
  if (s.flags & CCM_FLAG_NESTED) return make_plan_nested(s);
  if (s.flags & CCM_FLAG_SHARED_E) return make_plan_shared(s);

  Plan p;
  p.spec = s;
  p.mode = excl_mode(s.excl);
  p.window = s.excl > 0 ? s.excl : 0;
  const int nE = (int)s.E.size(), nT = (int)s.tau.size(), nL = (int)s.L.size();
  const int64_t N = s.N;
  p.n64 = 2 * N;
  p.n32 = 2 * N;
  p.ingest.push_back({0, 0, 2 * N});
  const int64_t sorted_limit = gather_max_sorted_n_e();
  p.n_out = 2LL * nE * nT * nL * s.r;
  p.L_eff.assign((size_t)nE * nT * nL, 0);

  for (int ie = 0; ie < nE; ++ie) {
    const int32_t E = s.E[ie];
    const int Q = crossmap_queries_per_lane(E);
    const int64_t qt = (int64_t)kBlock * Q;
    for (int it = 0; it < nT; ++it) {
      const int32_t tau = s.tau[it];
      const int64_t ne = N - (int64_t)(E - 1) * tau;
      int64_t emb_off[2], qord_off[2], ord_off[2];
      for (int sr = 0; sr < 2; ++sr) {
        emb_off[sr] = p.n_emb;
        qord_off[sr] = p.n_qord;
        ord_off[sr] = order_set(p, sr, embedding_order(E, tau));
        p.embed.push_back({sr * N, p.n_emb, ord_off[sr], p.n_qord, ne, N, E, tau});
        attach_kd(p, ord_off[sr], E, emb_off[sr], ne);
        p.n_emb += ne * E;
        p.n_qord += ne;
        p.max_embed = std::max(p.max_embed, ne * E);
      }
      const int32_t sorted = ne <= sorted_limit ? 1 : 0;
      if (sorted) p.max_sorted_n_e = std::max(p.max_sorted_n_e, ne);
      for (int il = 0; il < nL; ++il) {
        const int64_t le = std::min(s.L[il], ne);
        p.L_eff[((size_t)ie * nT + it) * nL + il] = le;
        for (int ri = 0; ri < s.r; ++ri) {
          const int64_t lib_off = p.n_lib;
          p.sample.push_back({s.seed, ne, le, lib_off, E, tau, ri, 0});
          p.n_lib += le;
          for (int dir = 0; dir < 2; ++dir) {
            // dir 0: library Y (series 1) predicts X (series 0); dir 1: reverse
            const int lib_s = dir == 0 ? 1 : 0;
            const int tgt_s = dir == 0 ? 0 : 1;
            Realization R{};
            R.emb_off = emb_off[lib_s];
            R.pts_off = p.n_pts;
            R.pj_off = p.n_pj;
            R.qord_off = qord_off[lib_s];
            R.tgt_off = tgt_s * N;
            R.E = E;
            R.tau = tau;
            R.n_e = (int32_t)ne;
            R.l_eff = (int32_t)le;
            R.n_query = (int32_t)(s.query_set ? le : ne);
            R.n_tiles = (int32_t)((R.n_query + qt - 1) / qt);
            R.slot_base = p.n_slots;
            R.out_index = ((((int64_t)dir * nE + ie) * nT + it) * nL + il) * s.r + ri;
            R.table_off = -1;
            if (use_table(p, E, ne, le)) {
              R.table_off = table_for(p, R.emb_off, ne, E);
              R.table_w = (int32_t)std::min<int64_t>(kTableWidth, ne);
              p.e_table_ne[E] = std::max(p.e_table_ne[E], (int)ne);
              p.table_rz += 1;
            }
            GatherJob gj{};
            gj.emb_off = R.emb_off;
            gj.lib_off = lib_off;
            gj.order_off = ord_off[lib_s];
            gj.pts_off = R.pts_off;
            gj.pj_off = R.pj_off;
            gj.start_off = R.slot_base * kWaves;
            gj.l_eff = le;
            gj.n_e = ne;
            gj.n_series = N;
            gj.E = E;
            gj.tau = tau;
            gj.qt = (int32_t)qt;
            gj.query_set = s.query_set;
            gj.sorted = sorted;
            p.gather.push_back(gj);
            p.n_pts += le * E;
            p.n_pj += le;
            p.n_slots += R.n_tiles;
            p.rz.push_back(R);
            p.rz_sample.push_back((int64_t)p.sample.size() - 1);
            p.rz_gather.push_back((int64_t)p.gather.size() - 1);
            // algorithmic work: every (query, candidate) pair but the query itself
            const double nq = (double)R.n_query;
            double pairs = nq * (double)le;
            if (p.mode == kExclSelf) pairs -= s.query_set ? nq : (double)le;
            p.pairs += pairs;
            p.flops += pairs * (3.0 * E - 1.0);
            p.preds += nq;
          }
        }
      }
    }
  }
  if (p.rz.size() > (size_t)INT32_MAX) fail(CCM_E_INVAL, "too many realizations");
  p.n_rho = (int64_t)p.rz.size();

  order_items(p);

  size_order_sort(p);
  p.device_bytes = p.n64 * 8 + p.n32 * 4 + p.n_emb * 4 + p.n_lib * 4 + p.n_pts * 4 +
                   p.n_pj * 4 + p.n_qord * 4 + p.n_slots * 4 * kWaves + p.sort_temp +
                   (size_t)p.n_ord * 16 + p.n_table * 4 + p.tables.size() * sizeof(TableJob) +
                   p.n_slots * sizeof(Moments) + p.n_out * 8 +
                   p.rz.size() * sizeof(Realization) + p.items.size() * sizeof(Item) +
                   p.sample.size() * sizeof(SampleJob) + p.gather.size() * sizeof(GatherJob);
  return p;
}

// Causal matrix: M series, one (E, tau); libraries per (L, r) shared by every
// series; one realization per (searched series, L, r) predicting all others.
Plan make_plan_matrix(const Spec& s) {
  if (s.M < 2) fail(CCM_E_INVAL, "M must be >= 2");
  if (s.flags & (CCM_FLAG_NESTED | CCM_FLAG_SHARED_E))
    fail(CCM_E_INVAL, "nested libraries and E-sweep sharing are not supported by the matrix form");
  if (s.N < 2) fail(CCM_E_INVAL, "N must be >= 2");
  if (s.L.empty()) fail(CCM_E_INVAL, "empty L list");
  if (s.r < 1) fail(CCM_E_INVAL, "r must be >= 1");
  if (s.query_set != 0 && s.query_set != 1) fail(CCM_E_INVAL, "query_set must be 0 or 1");
  // the kernel addresses the time-major target table (N rows of
  // target_stride(M) doubles) with 32-bit byte offsets
  if ((int64_t)target_stride(s.M) * s.N > ((int64_t)1 << 29))
    fail(CCM_E_INVAL, "M*N too large (the target table must stay within 4 GiB)");
  const int32_t E = s.E[0], tau = s.tau[0];
  if (E < 1 || E > kMaxE) fail(CCM_E_INVAL, "E must be in [1, 10]");
  if (tau < 1) fail(CCM_E_INVAL, "tau must be >= 1");
  const int64_t N = s.N;
  const int64_t ne = N - (int64_t)(E - 1) * tau;
  if (ne < E + 2) fail(CCM_E_INVAL, "N_e = N - (E-1) tau must be >= E + 2");
  for (int64_t l : s.L) {
    if (l < E + 2) fail(CCM_E_INVAL, "every L must be >= E + 2");
    if (std::min(l, ne) < min_library(E, s.excl))
      fail(CCM_E_INVAL, "library too small for the exclusion window");
  }
  Plan p;
  p.spec = s;
  p.mode = excl_mode(s.excl);
  p.window = s.excl > 0 ? s.excl : 0;
  const int M = s.M, nL = (int)s.L.size();
  p.n64 = (int64_t)M * N;
  p.n32 = (int64_t)M * N;
  p.ingest.push_back({0, 0, (int64_t)M * N});
  p.n_out = (int64_t)M * M * nL * s.r;
  p.L_eff.assign(nL, 0);
  const int Q = crossmap_queries_per_lane(E);
  const int64_t qt = (int64_t)kBlock * Q;
  const int32_t sorted = ne <= gather_max_sorted_n_e() ? 1 : 0;
  if (sorted) p.max_sorted_n_e = ne;
  std::vector<int64_t> emb_off(M), qord_off(M), ord_off(M);
  for (int a = 0; a < M; ++a) {
    emb_off[a] = p.n_emb;
    qord_off[a] = p.n_qord;
    ord_off[a] = order_set(p, a, embedding_order(E, tau));
    p.embed.push_back({a * N, p.n_emb, ord_off[a], p.n_qord, ne, N, E, tau});
    attach_kd(p, ord_off[a], E, emb_off[a], ne);
    p.n_emb += ne * E;
    p.n_qord += ne;
    p.max_embed = std::max(p.max_embed, ne * E);
  }
  std::vector<int64_t> lib_off((size_t)nL * s.r);
  for (int il = 0; il < nL; ++il) {
    const int64_t le = std::min(s.L[il], ne);
    p.L_eff[il] = le;
    for (int ri = 0; ri < s.r; ++ri) {
      lib_off[(size_t)il * s.r + ri] = p.n_lib;
      p.sample.push_back({s.seed, ne, le, p.n_lib, E, tau, ri, 0});
      p.n_lib += le;
    }
  }
  for (int a = 0; a < M; ++a)
    for (int il = 0; il < nL; ++il)
      for (int ri = 0; ri < s.r; ++ri) {
        const int64_t le = p.L_eff[il];
        Realization R{};
        R.emb_off = emb_off[a];
        R.pts_off = p.n_pts;
        R.pj_off = p.n_pj;
        R.qord_off = qord_off[a];
        R.tgt_off = 0;
        R.E = E;
        R.tau = tau;
        R.n_e = (int32_t)ne;
        R.l_eff = (int32_t)le;
        R.n_query = (int32_t)(s.query_set ? le : ne);
        R.n_tiles = (int32_t)((R.n_query + qt - 1) / qt);
        R.slot_base = p.n_slots;
        R.out_index = (((int64_t)a * M) * nL + il) * s.r + ri;   // target 0 of row a
        R.table_off = -1;
        if (use_table(p, E, ne, le)) {
          R.table_off = table_for(p, R.emb_off, ne, E);
          R.table_w = (int32_t)std::min<int64_t>(kTableWidth, ne);
          p.e_table_ne[E] = std::max(p.e_table_ne[E], (int)ne);
          p.table_rz += M - 1;   // rho values, like n_rho
        }
        GatherJob gj{};
        gj.emb_off = R.emb_off;
        gj.lib_off = lib_off[(size_t)il * s.r + ri];
        gj.order_off = ord_off[a];
        gj.pts_off = R.pts_off;
        gj.pj_off = R.pj_off;
        gj.start_off = R.slot_base * kWaves;
        gj.l_eff = le;
        gj.n_e = ne;
        gj.n_series = N;
        gj.E = E;
        gj.tau = tau;
        gj.qt = (int32_t)qt;
        gj.query_set = s.query_set;
        gj.sorted = sorted;
        p.gather.push_back(gj);
        p.n_pts += le * E;
        p.n_pj += le;
        p.n_slots += R.n_tiles;
        p.rz.push_back(R);
        p.self_of.push_back(a);
        p.rz_sample.push_back((int64_t)il * s.r + ri);
        p.rz_gather.push_back((int64_t)p.gather.size() - 1);
        const double nq = (double)R.n_query;
        double pairs = nq * (double)le;
        if (p.mode == kExclSelf) pairs -= s.query_set ? nq : (double)le;
        p.pairs += pairs;
        p.flops += pairs * (3.0 * E - 1.0);
        p.preds += nq * (M - 1);
      }
  p.n_rho = (int64_t)p.rz.size() * (M - 1);
  order_items(p);
  size_order_sort(p);
  p.device_bytes = p.n64 * 8 + p.n32 * 4 + p.n_ord * 16 + p.n_emb * 4 + p.n_lib * 4 +
                   p.n_pts * 4 +
                   p.n_pj * 4 + p.n_qord * 4 + p.n_slots * 4 * kWaves + p.sort_temp +
                   p.n_slots * M * multi_sums_bytes() + p.n_out * 8 +
                   N * target_stride(M) * 8 + p.n_table * 4 +
                   p.tables.size() * sizeof(TableJob) +
                   p.rz.size() * (sizeof(Realization) + 4) + p.items.size() * sizeof(Item) +
                   p.sample.size() * sizeof(SampleJob) + p.gather.size() * sizeof(GatherJob);
  return p;
}

void check_host_series(const double* s, int64_t n, const char* name) {
  if (!s) fail(CCM_E_INVAL, std::string(name) + " is NULL");
  for (int64_t t = 0; t < n; ++t)
    if (!std::isfinite(s[t]) || std::fabs(s[t]) > 1e17)
      fail(CCM_E_INVAL, std::string(name) + " has a non-finite or too large value");
}

Spec make_spec(int64_t N, const int32_t* E, int32_t nE, const int32_t* tau, int32_t ntau,
               const int64_t* L, int32_t nL, int32_t r, uint64_t seed,
               const ccm_opts* opts) {
  if (!E || !tau || !L) fail(CCM_E_INVAL, "NULL parameter array");
  if (nE < 1 || ntau < 1 || nL < 1) fail(CCM_E_INVAL, "nE, ntau and nL must be >= 1");
  Spec s;
  s.N = N;
  s.E.assign(E, E + nE);
  s.tau.assign(tau, tau + ntau);
  s.L.assign(L, L + nL);
  s.r = r;
  s.seed = seed;
  if (opts) {
    s.excl = opts->exclusion_radius;
    s.query_set = opts->query_set;
    s.flags = opts->flags;
  }
  return s;
}


}  // namespace ccmh
