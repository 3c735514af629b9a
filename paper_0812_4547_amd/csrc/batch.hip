// Batch plans: Algorithm 1 on many independent problems of different sizes
// with a fixed number of fused launches.
//
// Problems are grouped by the tile size their sketch uses (2^12..2^15, or the
// direct kernel for n' <= 2048).  Per pass the plan launches: the random
// streams of every problem (3 launches), per group the persistent sketch
// kernel over all (problem, column, tile) items of the group (tiles cut by
// row n included, with bounds-checked vector loads) and
// its reduce, the moments of every problem (2 launches), and
// Lawson-Hanson for every problem (one launch for d <= 64, one for d > 64;
// one wavefront per problem).  Descriptors of every problem live in device
// tables built once at plan time; the workspace is bound at plan time too, so
// a pass is a fixed sequence of launches that a HIP graph can replay.
//
// The autotuner times the sketch launches of the plan's own problems for
// each candidate (tile-size cap, workgroups per CU) and keeps the fastest.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

namespace {

using namespace rnnls;

struct Candidate {
  int log_t_cap, wgs;
};
// LDS bounds the occupancy: 2^15-row tiles use 132 KB of the 160 KB per CU.
const Candidate kCandidates[] = {{15, 1}, {14, 1}, {14, 2}, {13, 2}, {13, 3}, {13, 4}, {12, 4}, {12, 8}};
// row segments of a problem's moments at most (each at least 256 rows)
constexpr int kMomentSegments = 8;

// The autotuner's choices, process-wide, keyed by a plan's shapes.
struct TuneCache {
  std::mutex mu;
  std::map<uint64_t, Candidate> table;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

struct Settings {
  int sample_mode = RNNLS_SAMPLE_EXACT;
  int max_iter = 0;
  int r_cap = 0;
  double tol = 0.0;
};

// Rows the sketch buffers of one problem hold (a Bernoulli sample keeps at
// most n' rows, so the capacity is clamped to n').
int row_cap(int r, const Settings& o, int64_t n_pad) {
  if (o.sample_mode == RNNLS_SAMPLE_EXACT) return r;
  const int64_t want = o.r_cap > 0 ? o.r_cap : r + 8 * (int64_t)ceil(sqrt((double)r)) + 64;
  return (int)(want < n_pad ? want : n_pad);
}

int check_problem(const rnnls_problem& p, const Settings& o) {
  if (p.n < 2 || p.n > (1ll << 30)) return -1;
  if (p.d < 1 || p.d > RNNLS_MAX_D) return -1;
  const int64_t n_pad = (int64_t)next_pow2((uint64_t)p.n);
  if (p.r < 1 || (int64_t)p.r >= n_pad || p.r > RNNLS_MAX_R) return -1;
  const int rc = row_cap(p.r, o, n_pad);
  if (rc < 1 || rc > RNNLS_MAX_R) return -1;
  if (!p.A || p.lda < p.n || !p.b || !p.x) return -1;
  return 0;
}

struct Group {
  SrhtGroup g{};
  std::vector<int> members;  // problem indices
  std::vector<SketchJob> jobs;
  std::vector<int32_t> col_map;  // column of the group -> job in the group
  std::vector<int32_t> red_cols;  // columns of the group transformed by several workgroups
  SketchJob* dev = nullptr;
  int32_t* col_map_dev = nullptr;
  int32_t* red_cols_dev = nullptr;
};

}  // namespace

struct rnnls_batch {
  int count = 0;
  std::vector<rnnls_problem> probs;
  Settings opts;
  int cus = 0;
  Candidate tune{0, 0};  // 0 = the library's default choice
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device tables (one allocation)
  void* dev_tables = nullptr;
  std::vector<StreamJob> sjobs;
  StreamJob* sdev = nullptr;
  std::vector<int32_t> blk_map, chunk_map, ent_map;  // block -> job
  int32_t* blk_map_dev = nullptr;
  int32_t* chunk_map_dev = nullptr;
  int32_t* ent_map_dev = nullptr;
  std::vector<Group> groups;
  std::vector<MomentJob> mjobs;
  MomentJob* mdev = nullptr;
  int64_t m_chunks = 0;
  int m_max_pairs = 0;
  std::vector<LhJob> ljobs[2];  // d <= 64, d > 64
  LhJob* ldev[2] = {nullptr, nullptr};
  int l_max_d[2] = {0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the d <= 64 solves run on a second stream beside the d > 64 ones
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // learned proposal
  int64_t columns = 0;
  std::vector<char> fjobs;  // FeatJob records
  void* fdev = nullptr;
  float* X = nullptr;
  uint8_t* flags = nullptr;
  int32_t* warm_used = nullptr;
  const float* theta = nullptr;
  const uint16_t* wb = nullptr;
  float threshold = 0.5f;
};

namespace {

size_t put(size_t& off, size_t bytes) {
  const size_t at = off;
  off += align256(bytes);
  return at;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

bool aligned16(const void* p) { return ((uintptr_t)p % 16) == 0; }

// Workgroups per CU: the candidate's for the groups at its tile size, the
// default for groups whose n' or r forced another tile size.
int group_wgs(const Candidate& c, int log_t) {
  if (c.wgs > 0 && c.log_t_cap == log_t) return c.wgs;
  return srht_wgs_per_cu(log_t);
}

// Build every descriptor for candidate `c` laid out from ws (or only size the
// layout when ws is NULL).  Returns the workspace bytes.
size_t build(rnnls_batch& B, const Candidate& c, void* ws) {
  const int np = B.count;
  const Settings& o = B.opts;
  B.sjobs.assign(np, StreamJob{});
  B.mjobs.assign(np, MomentJob{});
  B.ljobs[0].clear();
  B.ljobs[1].clear();
  B.l_max_d[0] = B.l_max_d[1] = 0;
  B.groups.clear();

  // per-problem tile size and group
  std::vector<int> log_t(np), rcap(np), m(np);
  for (int i = 0; i < np; ++i) {
    const rnnls_problem& p = B.probs[i];
    m[i] = ilog2_exact(next_pow2((uint64_t)p.n));
    rcap[i] = row_cap(p.r, o, 1ll << m[i]);
    log_t[i] = srht_pref_log_t(m[i], rcap[i], c.log_t_cap);
  }
  const int group_keys[] = {15, 14, 13, 12, 0};
  for (int key : group_keys) {
    Group G;
    G.g.log_t = key;
    for (int i = 0; i < np; ++i)
      if (log_t[i] == key) G.members.push_back(i);
    if (!G.members.empty()) B.groups.push_back(std::move(G));
  }

  // grid of every group (needs the item count first)
  for (Group& G : B.groups) {
    int64_t items = 0, items_rag = 0, cols = 0;
    int max_rc = 0;
    bool vec = true;
    for (int i : G.members) {
      const rnnls_problem& p = B.probs[i];
      const int ncols = p.d + 1;
      if (G.g.log_t > 0)  // tiles cut by row n run in the same launch
        items += (int64_t)ncols * ((p.n + (1ll << G.g.log_t) - 1) >> G.g.log_t);
      cols += ncols;
      max_rc = std::max(max_rc, rcap[i]);
      vec = vec && aligned16(p.A) && p.lda % 4 == 0 && aligned16(p.b);
    }
    G.g.items = items;
    G.g.items_rag = items_rag;
    G.g.cols = cols;
    G.g.max_r_cap = max_rc;
    G.g.vec = vec;
    G.g.spt = G.g.log_t > 0 ? srht_spt(G.g.log_t, max_rc) : 0;
    const int64_t cap = (int64_t)B.cus * (G.g.log_t > 0 ? group_wgs(c, G.g.log_t) : 1);
    G.g.grid = (int)std::max<int64_t>(1, std::min(items, cap));
  }

  size_t off = 0;
  std::vector<size_t> o_rows(np), o_cnt(np), o_st(np), o_signs(np), o_scr(np), o_part(np),
      o_sa(np), o_sb(np), o_mom(np), o_G(np), o_q(np), o_c(np), o_abs(np);
  std::vector<int> pieces(np, 0);
  std::vector<MomentsPlan> mp(np);
  const int seg_cap = std::max(1, std::min(kMomentSegments, (4 * B.cus + np - 1) / np));
  // sketch items and pieces per group
  for (Group& G : B.groups) {
    int64_t item0 = 0, item0_rag = 0, col0 = 0;
    G.red_cols.clear();
    for (int i : G.members) {
      const rnnls_problem& p = B.probs[i];
      const int ncols = p.d + 1;
      SketchJob j{};
      j.n = p.n;
      j.d = p.d;
      j.ncols = ncols;
      j.r_cap = rcap[i];
      j.log_t = G.g.log_t;
      j.col0 = col0;
      col0 += ncols;
      if (G.g.log_t > 0) {
        j.tiles = (p.n + (1ll << G.g.log_t) - 1) >> G.g.log_t;
        j.rag = 0;
        j.item0 = item0;
        j.item0_rag = item0_rag;
        item0 += (int64_t)ncols * j.tiles;
        j.pieces = srht_owner_pieces(j.item0, j.tiles, ncols, G.g.items, G.g.grid);
        // only these columns have partials to add (the others are written
        // whole by the transform)
        for (int c = 0; c < ncols; ++c) {
          const int64_t first = j.item0 + (int64_t)c * j.tiles;
          if (srht_owner_of(first + j.tiles - 1, G.g.items, G.g.grid) !=
              srht_owner_of(first, G.g.items, G.g.grid))
            G.red_cols.push_back((int32_t)(j.col0 + c));
        }
      }
      pieces[i] = j.pieces;
      G.jobs.push_back(j);
    }
  }
  for (int i = 0; i < np; ++i) {
    const rnnls_problem& p = B.probs[i];
    const int64_t n_pad = 1ll << m[i];
    // row segments of at least 256 rows, at most 8 per problem, and no more
    // than about two workgroups per slot of the device (two per CU) over the
    // plan: a plan of thousands of problems fills the device with one segment
    // each and then writes no partial blocks (nor runs their reduce)
    mp[i] = moments_plan(rcap[i], p.d, 1, B.cus, seg_cap);
    o_rows[i] = put(off, sizeof(int32_t) * rcap[i]);
    o_cnt[i] = put(off, sizeof(int32_t));
    o_st[i] = put(off, sizeof(int32_t));
    o_signs[i] = put(off, sizeof(uint32_t) * (size_t)((n_pad + 31) / 32));
    o_scr[i] = put(off, sizeof(uint32_t) * streams_scratch_words(n_pad));
    o_part[i] = put(off, sizeof(float) * (size_t)(p.d + 1) * pieces[i] * rcap[i]);
    o_sa[i] = put(off, sizeof(float) * (size_t)p.d * rcap[i]);
    o_sb[i] = put(off, sizeof(float) * (size_t)rcap[i]);
    o_mom[i] = put(off, moments_scratch_bytes(mp[i]));
    o_G[i] = put(off, sizeof(double) * (size_t)p.d * p.d);
    o_q[i] = put(off, sizeof(double) * (size_t)p.d);
    o_c[i] = put(off, sizeof(double));
    o_abs[i] = put(off, sizeof(double) * (size_t)p.d);
  }
  int64_t columns = 0;
  for (int i = 0; i < np; ++i) columns += B.probs[i].d;
  const size_t o_X = put(off, sizeof(float) * (size_t)columns * RNNLS_MLP_FEATURES);
  const size_t o_fl = put(off, (size_t)columns);
  const size_t o_wu = put(off, sizeof(int32_t) * (size_t)np);
  const size_t total = off;
  if (!ws) return total;
  B.columns = columns;
  B.X = at<float>(ws, o_X);
  B.flags = at<uint8_t>(ws, o_fl);
  B.warm_used = at<int32_t>(ws, o_wu);
  B.fjobs.assign((size_t)np * feat_job_bytes(), 0);

  // fill pointers
  int64_t blk0 = 0, chunk0 = 0, row0 = 0;
  B.blk_map.clear();
  B.chunk_map.clear();
  B.ent_map.clear();
  int max_pairs = 0;
  for (int i = 0; i < np; ++i) {
    const rnnls_problem& p = B.probs[i];
    StreamJob& s = B.sjobs[i];
    s.seed = p.seed;
    s.m = m[i];
    s.r = p.r;
    s.r_cap = rcap[i];
    s.mode = o.sample_mode;
    s.sign_log_t = log_t[i];
    s.sign_rows = (int32_t)p.n;
    s.blk0 = blk0;
    blk0 += streams_blocks(m[i]);
    B.blk_map.insert(B.blk_map.end(), (size_t)streams_blocks(m[i]), i);
    s.sign_words = at<uint32_t>(ws, o_signs[i]);
    s.sign_export = nullptr;
    s.scratch = at<uint32_t>(ws, o_scr[i]);
    s.rows = at<int32_t>(ws, o_rows[i]);
    s.count = at<int32_t>(ws, o_cnt[i]);
    s.status = at<int32_t>(ws, o_st[i]);

    MomentJob& mj = B.mjobs[i];
    mj.M = at<float>(ws, o_sa[i]);
    mj.ldm = rcap[i];
    mj.F = at<float>(ws, o_sb[i]);
    mj.ldf = rcap[i];
    mj.m = rcap[i];
    mj.m_dev = s.count;
    mj.d = p.d;
    mj.k = 1;
    mj.chunks = mp[i].chunks;
    mj.nbA = mp[i].nbA;
    mj.nb = mp[i].nb;
    mj.pairs = mp[i].pairs;
    mj.chunk0 = chunk0;
    chunk0 += mp[i].chunks;
    B.chunk_map.insert(B.chunk_map.end(), (size_t)mp[i].chunks, i);
    mj.ent0 = (int64_t)B.ent_map.size() * 256;
    if (mp[i].chunks > 1)  // blocks of 256 reduce entries of this problem
      B.ent_map.insert(B.ent_map.end(), (size_t)((moments_entries(mp[i]) + 255) / 256), i);
    max_pairs = std::max(max_pairs, mp[i].pairs);
    double* scr = at<double>(ws, o_mom[i]);
    mj.part = scr;
    mj.part_abs = moments_abs_scratch(mp[i], scr);
    mj.G = at<double>(ws, o_G[i]);
    mj.Q = at<double>(ws, o_q[i]);
    mj.ldq = p.d;
    mj.c = at<double>(ws, o_c[i]);
    mj.colabs = at<double>(ws, o_abs[i]);

    LhJob lj{};
    lj.d = p.d;
    lj.max_iter = o.max_iter > 0 ? o.max_iter : 3 * p.d;
    lj.m = rcap[i];
    lj.tol = o.tol;
    lj.G = mj.G;
    lj.q = mj.Q;
    lj.c = mj.c;
    lj.colabs = mj.colabs;
    lj.m_dev = s.count;
    lj.pre_status = s.status;
    lj.x = p.x;
    lj.rnorm = p.rnorm;
    lj.iters = p.iters;
    lj.status = p.status;
    lj.theta = B.theta;
    lj.wb = B.wb;
    lj.threshold = B.threshold;
    lj.flags = B.theta ? B.flags + row0 : nullptr;
    lj.warm_used = B.warm_used + i;
    make_feat_job(B.fjobs.data() + (size_t)i * feat_job_bytes(), mj.G, mj.Q, mj.c, p.x, p.d,
                  row0);
    row0 += p.d;
    const int h = p.d > 64;
    B.ljobs[h].push_back(lj);
    B.l_max_d[h] = std::max(B.l_max_d[h], p.d);
  }
  // moments segments in decreasing order of work (block pairs x rows), so
  // that the launch ends on the short ones
  {
    std::vector<int> order(np);
    for (int i = 0; i < np; ++i) order[i] = i;
    auto work = [&](int i) {
      return (int64_t)B.mjobs[i].pairs * (B.mjobs[i].m / std::max(1, B.mjobs[i].chunks));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    int64_t c0 = 0;
    B.chunk_map.clear();
    for (int i : order) {
      B.mjobs[i].chunk0 = c0;
      c0 += B.mjobs[i].chunks;
      B.chunk_map.insert(B.chunk_map.end(), (size_t)B.mjobs[i].chunks, i);
    }
  }
  // widest problems first: a solve's time grows with d, and workgroups start
  // in launch order, so the short solves fill the launch's tail
  for (int h = 0; h < 2; ++h)
    std::stable_sort(B.ljobs[h].begin(), B.ljobs[h].end(),
                     [](const LhJob& a, const LhJob& b) { return a.d > b.d; });
  B.m_chunks = chunk0;
  B.m_max_pairs = max_pairs;
  for (Group& G : B.groups) {
    G.col_map.clear();
    for (size_t k = 0; k < G.members.size(); ++k) {
      const int i = G.members[k];
      const rnnls_problem& p = B.probs[i];
      SketchJob& j = G.jobs[k];
      G.col_map.insert(G.col_map.end(), (size_t)(p.d + 1), (int32_t)k);
      j.A = p.A;
      j.lda = p.lda;
      j.B = p.b;
      j.ldb = p.n;
      j.sign_words = B.sjobs[i].sign_words;
      j.rows = B.sjobs[i].rows;
      j.count = B.sjobs[i].count;
      j.partials = at<float>(ws, o_part[i]);
      j.SA = at<float>(ws, o_sa[i]);
      j.ldsa = rcap[i];
      j.SB = at<float>(ws, o_sb[i]);
      j.ldsb = rcap[i];
      j.inv_sqrt_r = 1.0 / sqrt((double)p.r);
    }
  }
  return total;
}

void free_streams(rnnls_batch& B) {
  if (B.fork) (void)hipEventDestroy(B.fork);
  if (B.join) (void)hipEventDestroy(B.join);
  if (B.side) (void)hipStreamDestroy(B.side);
  B.fork = B.join = nullptr;
  B.side = nullptr;
}

void free_tables(rnnls_batch& B) {
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  if (B.dev_tables) (void)hipFree(B.dev_tables);
  B.dev_tables = nullptr;
}

// Build for candidate c against the bound workspace and upload the tables.
int plan(rnnls_batch& B, const Candidate& c) {
  free_tables(B);
  const size_t need = build(B, c, nullptr);
  if (need > B.ws_bytes) return RNNLS_E_WORKSPACE;
  build(B, c, B.ws);
  size_t bytes = 0;
  const size_t o_s = bytes;
  bytes += align256(sizeof(StreamJob) * B.sjobs.size());
  std::vector<size_t> o_g;
  for (Group& G : B.groups) {
    o_g.push_back(bytes);
    bytes += align256(sizeof(SketchJob) * G.jobs.size());
  }
  const size_t o_m = bytes;
  bytes += align256(sizeof(MomentJob) * B.mjobs.size());
  size_t o_l[2];
  for (int h = 0; h < 2; ++h) {
    o_l[h] = bytes;
    bytes += align256(sizeof(LhJob) * B.ljobs[h].size());
  }
  const size_t o_f = bytes;
  bytes += align256(B.fjobs.size());
  auto map_bytes = [](const std::vector<int32_t>& v) { return align256(sizeof(int32_t) * v.size()); };
  const size_t o_bm = bytes;
  bytes += map_bytes(B.blk_map);
  const size_t o_cm = bytes;
  bytes += map_bytes(B.chunk_map);
  const size_t o_em = bytes;
  bytes += map_bytes(B.ent_map);
  std::vector<size_t> o_gm, o_rc;
  for (Group& G : B.groups) {
    o_gm.push_back(bytes);
    bytes += map_bytes(G.col_map);
    o_rc.push_back(bytes);
    bytes += map_bytes(G.red_cols);
  }
  if (hipMalloc(&B.dev_tables, bytes) != hipSuccess) {
    B.dev_tables = nullptr;
    return RNNLS_E_HIP;
  }
  std::vector<char> host(bytes, 0);
  auto copy = [&](size_t off, const void* src, size_t n) {
    if (n) memcpy(host.data() + off, src, n);
  };
  copy(o_s, B.sjobs.data(), sizeof(StreamJob) * B.sjobs.size());
  for (size_t g = 0; g < B.groups.size(); ++g)
    copy(o_g[g], B.groups[g].jobs.data(), sizeof(SketchJob) * B.groups[g].jobs.size());
  copy(o_m, B.mjobs.data(), sizeof(MomentJob) * B.mjobs.size());
  for (int h = 0; h < 2; ++h) copy(o_l[h], B.ljobs[h].data(), sizeof(LhJob) * B.ljobs[h].size());
  copy(o_f, B.fjobs.data(), B.fjobs.size());
  copy(o_bm, B.blk_map.data(), sizeof(int32_t) * B.blk_map.size());
  copy(o_cm, B.chunk_map.data(), sizeof(int32_t) * B.chunk_map.size());
  copy(o_em, B.ent_map.data(), sizeof(int32_t) * B.ent_map.size());
  for (size_t g = 0; g < B.groups.size(); ++g) {
    copy(o_gm[g], B.groups[g].col_map.data(), sizeof(int32_t) * B.groups[g].col_map.size());
    copy(o_rc[g], B.groups[g].red_cols.data(), sizeof(int32_t) * B.groups[g].red_cols.size());
  }
  if (hipMemcpy(B.dev_tables, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
    return RNNLS_E_HIP;
  char* base = static_cast<char*>(B.dev_tables);
  B.sdev = reinterpret_cast<StreamJob*>(base + o_s);
  for (size_t g = 0; g < B.groups.size(); ++g)
    B.groups[g].dev = reinterpret_cast<SketchJob*>(base + o_g[g]);
  B.mdev = reinterpret_cast<MomentJob*>(base + o_m);
  for (int h = 0; h < 2; ++h) B.ldev[h] = reinterpret_cast<LhJob*>(base + o_l[h]);
  B.fdev = base + o_f;
  B.blk_map_dev = reinterpret_cast<int32_t*>(base + o_bm);
  B.chunk_map_dev = reinterpret_cast<int32_t*>(base + o_cm);
  B.ent_map_dev = reinterpret_cast<int32_t*>(base + o_em);
  for (size_t g = 0; g < B.groups.size(); ++g) {
    B.groups[g].col_map_dev = reinterpret_cast<int32_t*>(base + o_gm[g]);
    B.groups[g].red_cols_dev = reinterpret_cast<int32_t*>(base + o_rc[g]);
  }
  B.tune = c;
  return RNNLS_OK;
}

int run_sketch(rnnls_batch& B, hipStream_t s) {
  for (Group& G : B.groups) {
    const int rc = launch_srht_batch(G.g, G.dev, (int)G.jobs.size(), G.col_map_dev,
                                     G.red_cols_dev, (int)G.red_cols.size(), s);
    if (rc) return rc;
  }
  return RNNLS_OK;
}

int run_all(rnnls_batch& B, hipStream_t s) {
  int rc = launch_streams_batch(B.sjobs.data(), B.sdev, B.count, B.blk_map_dev, s);
  if (rc) return rc;
  rc = run_sketch(B, s);
  if (rc) return rc;
  int max_cols = 0;
  for (int i = 0; i < B.count; ++i) max_cols = std::max(max_cols, B.probs[i].d + 1);
  rc = launch_moments_batch(B.mdev, B.count, max_cols, B.m_chunks, B.chunk_map_dev,
                            (int64_t)B.ent_map.size(), B.ent_map_dev, s);
  if (rc) return rc;
  // with a model, each Lawson-Hanson workgroup first computes its problem's
  // learned proposal (features and perceptron) and warm-starts from it.  The
  // two solve launches (d <= 64, d > 64) are independent: the smaller one
  // runs on the plan's second stream, forked from and joined back into `s`
  // (also inside a captured graph, as two branches).
  const bool model = B.theta != nullptr;
  const bool both = !B.ljobs[0].empty() && !B.ljobs[1].empty();
  if (both) {
    if (hipEventRecord(B.fork, s) != hipSuccess || hipStreamWaitEvent(B.side, B.fork, 0) != hipSuccess)
      return RNNLS_E_HIP;
    rc = launch_lawson_hanson_batch(B.ldev[0], (int)B.ljobs[0].size(), B.l_max_d[0], model,
                                    B.side);
    if (rc) return rc;
    if (hipEventRecord(B.join, B.side) != hipSuccess) return RNNLS_E_HIP;
    rc = launch_lawson_hanson_batch(B.ldev[1], (int)B.ljobs[1].size(), B.l_max_d[1], model, s);
    if (rc) return rc;
    return hipStreamWaitEvent(s, B.join, 0) == hipSuccess ? RNNLS_OK : RNNLS_E_HIP;
  }
  for (int h = 0; h < 2; ++h) {
    rc = launch_lawson_hanson_batch(B.ldev[h], (int)B.ljobs[h].size(), B.l_max_d[h], model, s);
    if (rc) return rc;
  }
  return RNNLS_OK;
}

Settings read_settings(const rnnls_opts* o) {
  Settings s;
  if (o) {
    s.sample_mode = o->sample_mode;
    s.max_iter = o->max_iter;
    s.r_cap = o->r_cap;
    s.tol = o->tol;
  }
  return s;
}

bool settings_valid(const rnnls_opts* o) {
  if (!o) return true;
  return (o->sample_mode == RNNLS_SAMPLE_EXACT || o->sample_mode == RNNLS_SAMPLE_BERNOULLI) &&
         o->precision == RNNLS_PREC_FP32;
}

// Key of a plan's shapes for the autotuner's cache: FNV-1a over the device's
// CU count, the sampling mode and every problem's (log2 n', d, row capacity).
uint64_t shape_key(const rnnls_batch& B) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xffu;
      h *= 0x100000001b3ull;
    }
  };
  mix((uint64_t)B.cus);
  mix((uint64_t)B.opts.sample_mode);
  mix((uint64_t)B.count);
  for (const rnnls_problem& p : B.probs) {
    mix((uint64_t)ilog2_exact(next_pow2((uint64_t)p.n)));
    mix((uint64_t)p.d);
    mix((uint64_t)row_cap(p.r, B.opts, (int64_t)next_pow2((uint64_t)p.n)));
  }
  return h;
}

}  // namespace

extern "C" {

size_t rnnls_batch_workspace_bytes(int32_t count, const rnnls_problem* probs,
                                   const rnnls_opts* opts) {
  if (count < 1 || !probs || !settings_valid(opts)) return 0;
  rnnls_batch B;
  B.count = count;
  B.probs.assign(probs, probs + count);
  B.opts = read_settings(opts);
  for (int i = 0; i < count; ++i)
    if (check_problem(B.probs[i], B.opts)) return 0;
  B.cus = device_cus();
  if (B.cus < 0) return 0;
  size_t most = build(B, Candidate{0, 0}, nullptr);
  for (const Candidate& c : kCandidates) most = std::max(most, build(B, c, nullptr));
  return most;
}

int rnnls_batch_create(rnnls_batch** out, int32_t count, const rnnls_problem* probs,
                       const rnnls_opts* opts, void* ws, size_t ws_bytes, int32_t* bad_index) {
  if (!out) return -1;
  *out = nullptr;
  if (count < 1) return -2;
  if (!probs) return -3;
  if (!settings_valid(opts)) return -4;
  rnnls_batch* B = new rnnls_batch();
  B->count = count;
  B->probs.assign(probs, probs + count);
  B->opts = read_settings(opts);
  for (int i = 0; i < count; ++i) {
    if (check_problem(B->probs[i], B->opts)) {
      if (bad_index) *bad_index = i;
      delete B;
      return -3;
    }
  }
  B->cus = device_cus();
  if (B->cus < 0) {
    const int rc = B->cus;
    delete B;
    return rc;
  }
  if (!ws || (uintptr_t)ws % 256 != 0) {
    delete B;
    return RNNLS_E_WORKSPACE;
  }
  B->ws = ws;
  B->ws_bytes = ws_bytes;
  int rc = RNNLS_OK;
  if (hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->join, hipEventDisableTiming) != hipSuccess)
    rc = RNNLS_E_HIP;
  if (rc == RNNLS_OK) rc = plan(*B, Candidate{0, 0});
  if (rc) {
    free_tables(*B);
    free_streams(*B);
    delete B;
    return rc;
  }
  *out = B;
  return RNNLS_OK;
}

int rnnls_batch_run(rnnls_batch* B, void* stream) {
  if (!B) return -1;
  return run_all(*B, reinterpret_cast<hipStream_t>(stream));
}

int rnnls_batch_autotune(rnnls_batch* B, void* stream, rnnls_tuning* chosen) {
  if (!B) return -1;
  const uint64_t key = shape_key(*B);
  {
    TuneCache& C = tune_cache();
    std::lock_guard<std::mutex> lock(C.mu);
    const auto it = C.table.find(key);
    if (it != C.table.end()) {  // the same shapes were timed before
      const int rc = plan(*B, it->second);
      if (rc) return rc;
      if (chosen) {
        chosen->srht_log_tile = it->second.log_t_cap;
        chosen->srht_wgs_per_cu = it->second.wgs;
      }
      return RNNLS_OK;
    }
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return RNNLS_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RNNLS_E_HIP;
  }
  int rc = RNNLS_OK;
  // the sketch of candidate c timed over `reps` launches (after one more),
  // in ms per launch; < 0 when the workspace cannot hold its layout
  auto time_candidate = [&](const Candidate& c, int reps, float* ms) -> int {
    *ms = -1.0f;
    int r = plan(*B, c);
    if (r == RNNLS_E_WORKSPACE) return RNNLS_OK;
    if (r) return r;
    // streams once (the sketch reads their output), then the sketch timed
    if ((r = launch_streams_batch(B->sjobs.data(), B->sdev, B->count, B->blk_map_dev, s)))
      return r;
    if ((r = run_sketch(*B, s))) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return RNNLS_E_HIP;
    for (int k = 0; k < reps && !r; ++k) r = run_sketch(*B, s);
    if (r) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return RNNLS_E_HIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return RNNLS_E_HIP;
    *ms = t / (float)reps;
    return RNNLS_OK;
  };
  // every candidate once, then the two fastest again in alternation (two
  // rounds): candidates within a few percent are told apart by the sum
  std::vector<std::pair<float, int>> timed;
  const int ncand = (int)(sizeof(kCandidates) / sizeof(kCandidates[0]));
  for (int ci = 0; ci < ncand && !rc; ++ci) {
    float ms = 0.0f;
    rc = time_candidate(kCandidates[ci], 3, &ms);
    if (!rc && ms >= 0.0f) timed.push_back({ms, ci});
  }
  std::sort(timed.begin(), timed.end());
  Candidate best_c{0, 0};
  if (!rc && !timed.empty()) {
    best_c = kCandidates[timed[0].second];
    if (timed.size() > 1) {
      float sum[2] = {timed[0].first, timed[1].first};
      for (int round = 0; round < 2 && !rc; ++round)
        for (int t = 0; t < 2 && !rc; ++t) {
          float ms = 0.0f;
          rc = time_candidate(kCandidates[timed[t].second], 3, &ms);
          sum[t] += ms;
        }
      if (!rc && sum[1] < sum[0]) best_c = kCandidates[timed[1].second];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int rc2 = plan(*B, best_c);
  if (rc) return rc;
  if (rc2) return rc2;
  {
    TuneCache& C = tune_cache();
    std::lock_guard<std::mutex> lock(C.mu);
    C.table[key] = best_c;
  }
  if (chosen) {
    chosen->srht_log_tile = best_c.log_t_cap;
    chosen->srht_wgs_per_cu = best_c.wgs;
  }
  return RNNLS_OK;
}

int rnnls_tuning_cache_entries(void) {
  TuneCache& C = tune_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  return (int)C.table.size();
}

int rnnls_tuning_cache_clear(void) {
  TuneCache& C = tune_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  C.table.clear();
  return RNNLS_OK;
}

int rnnls_tuning_cache_save(const char* path) {
  if (!path) return -1;
  TuneCache& C = tune_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  FILE* f = fopen(path, "w");
  if (!f) return RNNLS_E_UNSUPPORTED;
  bool ok = true;
  for (const auto& e : C.table)
    ok = ok && fprintf(f, "%016llx %d %d\n", (unsigned long long)e.first, e.second.log_t_cap,
                       e.second.wgs) > 0;
  ok = (fclose(f) == 0) && ok;
  return ok ? RNNLS_OK : RNNLS_E_UNSUPPORTED;
}

int rnnls_tuning_cache_load(const char* path) {
  if (!path) return -1;
  FILE* f = fopen(path, "r");
  if (!f) return RNNLS_E_UNSUPPORTED;
  std::map<uint64_t, Candidate> read;
  unsigned long long key = 0;
  int lt = 0, w = 0;
  int got;
  while ((got = fscanf(f, "%llx %d %d", &key, &lt, &w)) == 3) {
    bool known = false;
    for (const Candidate& c : kCandidates) known = known || (c.log_t_cap == lt && c.wgs == w);
    known = known || (lt == 0 && w == 0);
    if (!known) break;
    read[(uint64_t)key] = Candidate{lt, w};
  }
  const bool ok = got == EOF && feof(f);
  fclose(f);
  if (!ok) return RNNLS_E_UNSUPPORTED;  // nothing merged from a malformed file
  TuneCache& C = tune_cache();
  std::lock_guard<std::mutex> lock(C.mu);
  for (const auto& e : read) C.table[e.first] = e.second;
  return RNNLS_OK;
}

int rnnls_batch_capture(rnnls_batch* B) {
  if (!B) return -1;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return RNNLS_E_HIP;
  int rc = RNNLS_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
    rc = RNNLS_E_HIP;
  } else {
    rc = run_all(*B, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc == RNNLS_OK && (e != hipSuccess || !g)) rc = RNNLS_E_HIP;
    if (rc == RNNLS_OK) {
      if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        B->exec = nullptr;
        rc = RNNLS_E_HIP;
      }
    }
    if (rc == RNNLS_OK) B->graph = g;
    else if (g) (void)hipGraphDestroy(g);
  }
  (void)hipStreamDestroy(cs);
  return rc;
}

int rnnls_batch_launch(rnnls_batch* B, void* stream) {
  if (!B) return -1;
  if (!B->exec) return RNNLS_E_UNSUPPORTED;
  return hipGraphLaunch(B->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? RNNLS_OK
             : RNNLS_E_HIP;
}

int rnnls_batch_columns(const rnnls_batch* B, int64_t* columns) {
  if (!B) return -1;
  if (!columns) return -2;
  *columns = B->columns;
  return RNNLS_OK;
}

int rnnls_batch_features(rnnls_batch* B, float* X, uint8_t* passive, void* stream) {
  if (!B) return -1;
  if (!X) return -2;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = launch_features_batch(B->fdev, B->count, X, s);
  if (rc == RNNLS_OK && passive) rc = launch_passive_flags(B->fdev, B->count, passive, s);
  return rc;
}

int rnnls_batch_set_model(rnnls_batch* B, const float* theta, const uint16_t* wb,
                          float threshold) {
  if (!B) return -1;
  if (theta && !wb) return -3;
  if (wb && (uintptr_t)wb % 4 != 0) return -3;
  if (!(threshold > 0.0f && threshold < 1.0f)) return -4;
  B->theta = theta;
  B->wb = wb;
  B->threshold = threshold;
  return plan(*B, B->tune);  // the Lawson-Hanson descriptors gain or lose the model
}

int rnnls_batch_warm_used(rnnls_batch* B, int32_t* out, void* stream) {
  if (!B) return -1;
  if (!out) return -2;
  return hipMemcpyAsync(out, B->warm_used, sizeof(int32_t) * B->count, hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? RNNLS_OK
             : RNNLS_E_HIP;
}

int rnnls_batch_proposal(rnnls_batch* B, uint8_t* out, void* stream) {
  if (!B) return -1;
  if (!out) return -2;
  if (B->columns < 1) return RNNLS_OK;
  return hipMemcpyAsync(out, B->flags, (size_t)B->columns, hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? RNNLS_OK
             : RNNLS_E_HIP;
}

int rnnls_batch_destroy(rnnls_batch* B) {
  if (!B) return RNNLS_OK;
  const bool ok = hipDeviceSynchronize() == hipSuccess;
  free_tables(*B);
  free_streams(*B);
  delete B;
  return ok ? RNNLS_OK : RNNLS_E_HIP;
}

}  // extern "C"
