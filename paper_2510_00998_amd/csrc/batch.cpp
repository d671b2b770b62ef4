// Batched solver: many independent problems (each built by hpmg_setup with
// its own mesh, degree and max_rhs) solved together.  Every phase of the hp
// V-cycle runs as one persistent launch over a work list that covers every
// problem and right-hand side at that level; one iteration of the FP64
// flexible CG (FP32 V-cycle inside) is captured once as a HIP graph and
// replayed.  The persistent grid size, one launch per degree or one for all,
// and the cells per block of each degree (tile variant) are chosen by timing
// the V-cycle (autotuning) at the first solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"

using namespace hpmg::detail;

namespace {

struct Launch {
  int kind = 0;  // 0: DG float, 1: DG double, 2: Q1 float
  int op = 0;
  const void* args = nullptr;
  const hpmg::WorkItem* items = nullptr;  // DG: sorted by degree; cell blocks of tile variant 0
  int nitems = 0;
  // DG: runs of equal degree in `items` (degree, first item, count)
  std::vector<int3> runs;
  // DG: the same work in the cell blocks of tile variant 1 (half the cells
  // per block), for the one-launch-per-degree kernels
  const hpmg::WorkItem* items1 = nullptr;
  std::vector<int3> runs1;
};

// Items sorted by degree (stable), uploaded to mem, and their degree runs.
const hpmg::WorkItem* sorted_runs(DevMem& mem, std::vector<hpmg::WorkItem> items, std::vector<int3>& runs,
                                  hipStream_t s) {
  std::stable_sort(items.begin(), items.end(),
                   [](const hpmg::WorkItem& a, const hpmg::WorkItem& b) { return a.w < b.w; });
  for (int i = 0; i < (int)items.size(); ++i) {
    if (runs.empty() || runs.back().x != items[i].w) runs.push_back(int3{items[i].w, i, 0});
    ++runs.back().z;
  }
  return mem.upload(items, s);
}

// DG launch over `items` (tile variant 0) and `items1` (the same work in
// tile variant 1).
Launch dg_launch(DevMem& mem, int kind, int op, const void* args, std::vector<hpmg::WorkItem> items,
                 std::vector<hpmg::WorkItem> items1, hipStream_t s) {
  Launch L;
  L.kind = kind;
  L.op = op;
  L.args = args;
  L.nitems = (int)items.size();
  if (items.empty()) return L;
  L.items = sorted_runs(mem, std::move(items), L.runs, s);
  L.items1 = sorted_runs(mem, std::move(items1), L.runs1, s);
  return L;
}

}  // namespace

// Everything that depends on the number of right-hand sides: workspace,
// segment tables, launch lists and the captured iteration.
struct BatchPlan {
  int nrhs = 0;
  bool split = true;         // one launch per degree (tuned with the grid)
  int tile = 0;              // bit N: degree-N launches use tile variant 1 (tuned after the grid)
  std::vector<size_t> off0;  // offset of each problem in the workspace vectors
  size_t total = 0;          // their length
  int grid = 0;  // persistent grid (blocks) of the batched launches, 0: not tuned
  DevMem mem;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
  double *partial = nullptr, *scal = nullptr;
  int* count = nullptr;
  hpmg::SegTable seg{};
  double** seg_u = nullptr;  // device tables of the caller's vectors, set per call
  const double** seg_b = nullptr;
  std::vector<Launch> vcycle, applyp;
  Launch proj_u, resid_r, resid_z;  // projection of u; b - A u into r or into z
  hpmg::DGArgs<double>* resid_args = nullptr;
  std::vector<hpmg::DGArgs<double>> resid_args_h;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // level-0 smoothing of the caller's vectors (hpmg_batch_smooth), per
  // dtype: argument table [projection | even sweep | odd sweep] x problems
  // whose u, b are set per call through a pinned staging copy
  struct Smooth {
    void* args = nullptr;
    void* host = nullptr;
    size_t bytes = 0;
    Launch proj, even, odd;
    int grid = 0;
    bool split = true;
    int tile = 0;
    hipEvent_t copied = nullptr;  // the last staging copy has completed
  } sm[2];
  ~BatchPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto& S : sm) {
      if (S.copied) (void)hipEventDestroy(S.copied);
      if (S.host) (void)hipHostFree(S.host);
    }
  }
};

struct hpmg_batch_ctx {
  std::vector<hpmg_handle> hs;
  hipStream_t st = nullptr;
  int* host_count = nullptr;  // pinned
  std::unique_ptr<BatchPlan> plan;
  ~hpmg_batch_ctx() {
    plan.reset();
    if (host_count) (void)hipHostFree(host_count);
    if (st) (void)hipStreamDestroy(st);
  }
};

namespace {

template <typename T>
struct Table {
  std::vector<T> args;
  std::vector<hpmg::WorkItem> items;   // cell blocks of tile variant 0
  std::vector<hpmg::WorkItem> items1;  // of tile variant 1 (DG only)
};

int cpb_of(int N, int V) { return hpmg::cells_per_block_v(3, N, V); }

// Launch builder: collects per-problem arguments and work items, uploads.
struct Builder {
  BatchPlan* b;
  hipStream_t s;
  template <typename T>
  Launch dg(int op, Table<hpmg::DGArgs<T>>& t) {
    if (t.items.empty()) return Launch{};
    return dg_launch(b->mem, sizeof(T) == 4 ? 0 : 1, op, b->mem.upload(t.args, s), t.items, t.items1, s);
  }
  Launch cg(Table<hpmg::CGArgs<float>>& t) {
    Launch L;
    L.kind = 2;
    if (t.items.empty()) return L;
    L.args = b->mem.upload(t.args, s);
    L.items = b->mem.upload(t.items, s);
    L.nitems = (int)t.items.size();
    return L;
  }
};

template <typename T>
void add_dg_items(Table<hpmg::DGArgs<T>>& t, const hpmg::DGArgs<T>& a, int N, int nrhs) {
  const int idx = (int)t.args.size();
  t.args.push_back(a);
  for (int V = 0; V < hpmg::kTileVariants; ++V) {
    const int nb = (a.ncell + cpb_of(N, V) - 1) / cpb_of(N, V);
    for (int r = 0; r < nrhs; ++r)
      for (int blk = 0; blk < nb; ++blk) (V == 0 ? t.items : t.items1).push_back(hpmg::WorkItem{idx, blk, r, N});
  }
}

void add_cg_items(Table<hpmg::CGArgs<float>>& t, const hpmg::CGArgs<float>& a, int count, int nrhs) {
  const int idx = (int)t.args.size();
  t.args.push_back(a);
  const int nb = (count + 255) / 256;
  for (int r = 0; r < nrhs; ++r)
    for (int blk = 0; blk < nb; ++blk) t.items.push_back(hpmg::WorkItem{idx, blk, r, 0});
}

// Per-problem cursor through the V-cycle schedule.
struct PState {
  int ndg = 0, ncg = 0;
  std::vector<int> dgcur, cgcur;  // current trace buffer / current Q1 iterate
};

// FP32 V-cycle of every problem with a zero initial guess on level 0
// (u = z32 segment, b = r32 segment), as a list of batched launches.
void build_vcycle(BatchPlan* B, const std::vector<hpmg_handle>& hs, const std::vector<size_t>& off0, hipStream_t s) {
  Builder bld{B, s};
  const int R = B->nrhs;
  const int np = (int)hs.size();
  std::vector<PState> ps(np);
  int lmax = 0;
  for (int j = 0; j < np; ++j) {
    ps[j].ndg = (int)hs[j]->dg.size();
    ps[j].ncg = (int)hs[j]->cg.size();
    ps[j].dgcur.assign(ps[j].ndg, 0);
    ps[j].cgcur.assign(ps[j].ncg, 0);
    lmax = std::max(lmax, ps[j].ndg + ps[j].ncg);
  }
  const hpmg_options& O = hs[0]->opt;
  const int cg_pre = O.nu_pre_cg >= 0 ? O.nu_pre_cg : O.nu_pre;
  const int cg_post = O.nu_post_cg >= 0 ? O.nu_post_cg : O.nu_post;
  // level-l vectors of problem j
  auto dg_u = [&](int j, int l) -> float* { return l == 0 ? B->z32 + off0[j] : hs[j]->dg[l].f.u; };
  auto dg_b = [&](int j, int l) -> float* { return l == 0 ? B->r32 + off0[j] : hs[j]->dg[l].f.b; };

  std::vector<Launch>& out = B->vcycle;
  // recursive descent over the level index
  std::function<void(int)> rec = [&](int l) {
    std::vector<int> P;
    for (int j = 0; j < np; ++j)
      if (l < ps[j].ndg + ps[j].ncg) P.push_back(j);
    if (P.empty()) return;
    auto is_dg = [&](int j) { return l < ps[j].ndg; };
    auto cgl = [&](int j) { return l - ps[j].ndg; };
    auto coarsest = [&](int j) { return !is_dg(j) && cgl(j) == ps[j].ncg - 1; };
    // coarsest levels: dense solve
    {
      Table<hpmg::CGArgs<float>> t;
      for (int j : P)
        if (coarsest(j)) {
          hpmg_ctx* h = hs[j];
          CGLevel& C = h->cg[cgl(j)];
          hpmg::CGArgs<float> a{};
          a.op = hpmg::CGOP_DENSE;
          a.m = h->coarse_m;
          a.Ainv = h->coarse_inv;
          a.in = C.f.b;
          a.out = C.f.u[0];
          a.sin = a.sout = (long long)C.size;
          ps[j].cgcur[cgl(j)] = 0;
          add_cg_items(t, a, a.m, R);
        }
      Launch L = bld.cg(t);
      if (L.nitems) out.push_back(L);
    }
    // pre-smoothing (DG and Q1 levels each take their own count)
    for (int i = 0; i < std::max(O.nu_pre, cg_pre); ++i) {
      Table<hpmg::DGArgs<float>> td;
      Table<hpmg::CGArgs<float>> tc;
      for (int j : P) {
        hpmg_ctx* h = hs[j];
        if (is_dg(j) ? i >= O.nu_pre : i >= cg_pre) continue;
        if (is_dg(j)) {
          DGLevel& L = h->dg[l];
          int& cur = ps[j].dgcur[l];
          hpmg::DGArgs<float> a = dg_args<float>(h, L);
          a.u_in = a.u_out = dg_u(j, l);
          a.b = dg_b(j, l);
          a.tr_in = L.f.tr[cur];
          a.tr_out = L.f.tr[cur ^ 1];
          cur ^= 1;
          add_dg_items(td, a, L.N, R);
        } else if (!coarsest(j)) {
          CGLevel& C = h->cg[cgl(j)];
          int& cur = ps[j].cgcur[cgl(j)];
          hpmg::CGArgs<float> a{};
          a.op = hpmg::CGOP_JACOBI;
          a.nv = C.nv;
          a.uzero = i == 0;
          a.omega = (float)O.omega_cg;
          a.st = C.f.st;
          a.dinv = C.f.dinv;
          a.u = C.f.u[cur];
          a.b = C.f.b;
          a.out = C.f.u[cur ^ 1];
          a.su = a.sb = a.sout = (long long)C.size;
          cur ^= 1;
          add_cg_items(tc, a, (int)C.size, R);
        }
      }
      Launch L1 = bld.dg<float>(i == 0 ? hpmg::BOP_SWEEP0 : hpmg::BOP_SWEEP, td);
      if (L1.nitems) out.push_back(L1);
      Launch L2 = bld.cg(tc);
      if (L2.nitems) out.push_back(L2);
    }
    // residual and restriction
    {
      Table<hpmg::DGArgs<float>> td;
      Table<hpmg::CGArgs<float>> tg, tr, tre;
      for (int j : P) {
        hpmg_ctx* h = hs[j];
        if (is_dg(j)) {
          DGLevel& L = h->dg[l];
          hpmg::DGArgs<float> a = dg_args<float>(h, L);
          a.u_in = dg_u(j, l);
          a.b = dg_b(j, l);
          a.tr_in = L.f.tr[ps[j].dgcur[l]];
          if (!L.next_cg) {
            a.out = h->dg[l + 1].f.b;
            a.cstride = (long long)h->dg[l + 1].ndof;
          } else {
            a.out = L.f.contrib;
            a.cstride = (long long)h->ncell << 3;
            CGLevel& C = h->cg[0];
            hpmg::CGArgs<float> g{};
            g.op = hpmg::CGOP_GATHER;
            g.n = h->n;
            g.in = L.f.contrib;
            g.out = C.f.b;
            g.sin = (long long)h->ncell << 3;
            g.sout = (long long)C.size;
            add_cg_items(tg, g, (int)C.size, R);
          }
          add_dg_items(td, a, L.N, R);
        } else if (!coarsest(j)) {
          CGLevel& C = h->cg[cgl(j)];
          CGLevel& Cc = h->cg[cgl(j) + 1];
          hpmg::CGArgs<float> a{};
          a.op = hpmg::CGOP_RESID;
          a.nv = C.nv;
          a.st = C.f.st;
          a.u = C.f.u[ps[j].cgcur[cgl(j)]];
          a.b = C.f.b;
          a.out = C.f.r;
          a.su = a.sb = a.sout = (long long)C.size;
          add_cg_items(tr, a, (int)C.size, R);
          hpmg::CGArgs<float> rr{};
          rr.op = hpmg::CGOP_RESTRICT;
          rr.nv = C.nv;
          rr.nvc = Cc.nv;
          rr.idx = C.ridx;
          rr.w = C.f.rw;
          rr.in = C.f.r;
          rr.out = Cc.f.b;
          rr.sin = (long long)C.size;
          rr.sout = (long long)Cc.size;
          add_cg_items(tre, rr, (int)Cc.size, R);
        }
      }
      Launch L1 = bld.dg<float>(hpmg::BOP_RESTRICT, td);
      if (L1.nitems) out.push_back(L1);
      Launch L2 = bld.cg(tg);
      if (L2.nitems) out.push_back(L2);
      Launch L3 = bld.cg(tr);
      if (L3.nitems) out.push_back(L3);
      Launch L4 = bld.cg(tre);
      if (L4.nitems) out.push_back(L4);
    }
    rec(l + 1);
    // prolongation
    {
      Table<hpmg::DGArgs<float>> td;
      Table<hpmg::CGArgs<float>> tc;
      for (int j : P) {
        if (coarsest(j)) continue;
        hpmg_ctx* h = hs[j];
        if (is_dg(j)) {
          DGLevel& L = h->dg[l];
          hpmg::DGArgs<float> a = dg_args<float>(h, L);
          a.u_in = a.u_out = dg_u(j, l);
          a.tr_out = L.f.tr[ps[j].dgcur[l]];
          if (!L.next_cg) {
            a.coarse = h->dg[l + 1].f.u;
            a.coarse_cg = 0;
            a.cstride = (long long)h->dg[l + 1].ndof;
          } else {
            a.coarse = h->cg[0].f.u[ps[j].cgcur[0]];
            a.coarse_cg = 1;
            a.cstride = (long long)h->cg[0].size;
          }
          add_dg_items(td, a, L.N, R);
        } else {
          CGLevel& C = h->cg[cgl(j)];
          CGLevel& Cc = h->cg[cgl(j) + 1];
          hpmg::CGArgs<float> a{};
          a.op = hpmg::CGOP_PROLONG;
          a.nv = C.nv;
          a.nvc = Cc.nv;
          a.idx = C.pidx;
          a.w = C.f.pw;
          a.in = Cc.f.u[ps[j].cgcur[cgl(j) + 1]];
          a.out = C.f.u[ps[j].cgcur[cgl(j)]];
          a.sin = (long long)Cc.size;
          a.sout = (long long)C.size;
          add_cg_items(tc, a, (int)C.size, R);
        }
      }
      Launch L1 = bld.dg<float>(hpmg::BOP_PROLONG, td);
      if (L1.nitems) out.push_back(L1);
      Launch L2 = bld.cg(tc);
      if (L2.nitems) out.push_back(L2);
    }
    // post-smoothing
    for (int i = 0; i < std::max(O.nu_post, cg_post); ++i) {
      Table<hpmg::DGArgs<float>> td;
      Table<hpmg::CGArgs<float>> tc;
      for (int j : P) {
        if (coarsest(j)) continue;
        if (is_dg(j) ? i >= O.nu_post : i >= cg_post) continue;
        hpmg_ctx* h = hs[j];
        if (is_dg(j)) {
          DGLevel& L = h->dg[l];
          int& cur = ps[j].dgcur[l];
          hpmg::DGArgs<float> a = dg_args<float>(h, L);
          a.u_in = a.u_out = dg_u(j, l);
          a.b = dg_b(j, l);
          a.tr_in = L.f.tr[cur];
          a.tr_out = L.f.tr[cur ^ 1];
          cur ^= 1;
          add_dg_items(td, a, L.N, R);
        } else {
          CGLevel& C = h->cg[cgl(j)];
          int& cur = ps[j].cgcur[cgl(j)];
          hpmg::CGArgs<float> a{};
          a.op = hpmg::CGOP_JACOBI;
          a.nv = C.nv;
          a.uzero = 0;
          a.omega = (float)O.omega_cg;
          a.st = C.f.st;
          a.dinv = C.f.dinv;
          a.u = C.f.u[cur];
          a.b = C.f.b;
          a.out = C.f.u[cur ^ 1];
          a.su = a.sb = a.sout = (long long)C.size;
          cur ^= 1;
          add_cg_items(tc, a, (int)C.size, R);
        }
      }
      Launch L1 = bld.dg<float>(hpmg::BOP_SWEEP, td);
      if (L1.nitems) out.push_back(L1);
      Launch L2 = bld.cg(tc);
      if (L2.nitems) out.push_back(L2);
    }
  };
  rec(0);
}

// One-degree launch of a degree run in tile variant V.
template <typename T>
void dg_run(int V, int op, const int3& r, const void* args, const hpmg::WorkItem* items, int grid, hipStream_t s) {
  if (V == 0)
    hpmg::batch_dg_n_t0<T>(op, r.x, (const hpmg::DGArgs<T>*)args, items + r.y, r.z, grid, s);
  else
    hpmg::batch_dg_n_t1<T>(op, r.x, (const hpmg::DGArgs<T>*)args, items + r.y, r.z, grid, s);
}

// split: one launch per degree run (each with its own kernel; degree N in
// tile variant (tile >> N) & 1), else one launch over all degrees
void run_grid(const std::vector<Launch>& v, int grid, bool split, int tile, hipStream_t s) {
  for (const Launch& L : v) {
    if (L.nitems == 0) continue;
    if (L.kind == 2) {
      hpmg::batch_cg<float>((const hpmg::CGArgs<float>*)L.args, L.items, L.nitems, grid, s);
    } else if (split) {
      for (int V = 0; V < hpmg::kTileVariants; ++V)
        for (const int3& r : V == 0 ? L.runs : L.runs1) {
          if (((tile >> r.x) & 1) != V) continue;
          if (L.kind == 0)
            dg_run<float>(V, L.op, r, L.args, V == 0 ? L.items : L.items1, grid, s);
          else
            dg_run<double>(V, L.op, r, L.args, V == 0 ? L.items : L.items1, grid, s);
        }
    } else if (L.kind == 0) {
      hpmg::batch_dg<float>(L.op, (const hpmg::DGArgs<float>*)L.args, L.items, L.nitems, grid, s);
    } else {
      hpmg::batch_dg<double>(L.op, (const hpmg::DGArgs<double>*)L.args, L.items, L.nitems, grid, s);
    }
  }
  HIPCHK(hipGetLastError());
}

void run(BatchPlan* B, const std::vector<Launch>& v, hipStream_t s) {
  run_grid(v, B->grid > 0 ? B->grid : 1024, B->split, B->tile, s);  // before tuning: a default
}

// One iteration of the flexible CG for every segment; r32 holds r cast to
// FP32 (scale s[14]) on entry and on exit.
void iteration(BatchPlan* B, hipStream_t s) {
  const hpmg::SegTable& t = B->seg;
  run(B, B->vcycle, s);                                         // z32 = M r32
  hpmg::bk_dot_z(t, B->z32, B->r, B->q, B->scal, B->partial, s);  // z.r, z.q_old
  hpmg::bk_finalize(t, 1, B->partial, B->scal, 0.0, s);         // beta, rho
  hpmg::bk_update_p(t, B->z32, B->p, B->scal, s);               // p = z + beta p
  run(B, B->applyp, s);                                         // q = A p
  hpmg::bk_dot(t, B->p, B->q, nullptr, B->partial, s);
  hpmg::bk_finalize(t, 2, B->partial, B->scal, 0.0, s);         // alpha
  hpmg::bk_update_ur(t, B->r, B->r32, B->p, B->q, B->scal, B->partial, s);
  hpmg::bk_finalize(t, 3, B->partial, B->scal, 0.0, s);         // r.r, convergence (rtol^2 from scal)
  hpmg::bk_count(t, B->scal, B->count, s);
  HIPCHK(hipGetLastError());
}

// b - A u of the caller's vectors (FP64) into r (into_z = false) or z
void residual(BatchPlan* B, bool into_z, hipStream_t s) {
  run(B, {B->proj_u, into_z ? B->resid_z : B->resid_r}, s);
}

// Workspace, segment tables and launch lists for nrhs right-hand sides.
std::unique_ptr<BatchPlan> make_plan(const std::vector<hpmg_handle>& hs, int nrhs, hipStream_t s) {
  std::unique_ptr<BatchPlan> B(new BatchPlan());
  // the batch workspace comes from the first handle's allocator
  B->mem.alloc_fn = hs[0]->opt.alloc;
  B->mem.free_fn = hs[0]->opt.free;
  B->mem.ctx = hs[0]->opt.alloc_ctx;
  B->nrhs = nrhs;
  const int np = (int)hs.size(), R = nrhs;
  // segments: one per (problem, right-hand side), [problem][rhs][dof] in
  // the workspace vectors
  std::vector<size_t> off0(np);
  std::vector<long long> seg_off;
  std::vector<int> seg_len, cstart, ccount;
  std::vector<int2> chunks;
  size_t tot = 0;
  for (int j = 0; j < np; ++j) {
    off0[j] = tot;
    const size_t nd = hs[j]->ndof;
    for (int r = 0; r < R; ++r) {
      seg_off.push_back((long long)(tot + r * nd));
      seg_len.push_back((int)nd);
      cstart.push_back((int)chunks.size());
      int cnt = 0;
      for (size_t e = 0; e < nd; e += hpmg::BATCH_CHUNK, ++cnt)
        chunks.push_back(int2{(int)seg_off.size() - 1, (int)e});
      ccount.push_back(cnt);
    }
    tot += nd * R;
  }
  B->off0 = off0;
  B->total = tot;
  DevMem& M = B->mem;
  B->r = (double*)M.alloc(tot * sizeof(double));
  B->z = (double*)M.alloc(tot * sizeof(double));
  B->p = (double*)M.alloc(tot * sizeof(double));
  B->q = (double*)M.alloc(tot * sizeof(double));
  B->r32 = (float*)M.alloc(tot * sizeof(float));
  B->z32 = (float*)M.alloc(tot * sizeof(float));
  const int nseg = (int)seg_off.size();
  B->partial = (double*)M.alloc(2 * chunks.size() * sizeof(double));
  B->scal = (double*)M.alloc((size_t)nseg * hpmg::BATCH_SCAL * sizeof(double));
  B->count = (int*)M.alloc(4 * sizeof(int));
  B->seg.off = M.upload(seg_off, s);
  B->seg.len = M.upload(seg_len, s);
  B->seg.chunks = M.upload(chunks, s);
  B->seg.cstart = M.upload(cstart, s);
  B->seg.ccount = M.upload(ccount, s);
  B->seg.nseg = nseg;
  B->seg.nchunks = (int)chunks.size();
  B->seg_u = (double**)M.alloc(nseg * sizeof(double*));
  B->seg_b = (const double**)M.alloc(nseg * sizeof(double*));
  B->seg.u = B->seg_u;
  B->seg.b = B->seg_b;
  // FP32 V-cycle of every problem
  build_vcycle(B.get(), hs, off0, s);
  // FP64 q = A p (projection, then apply) and b - A u of the caller's vectors
  Builder bld{B.get(), s};
  Table<hpmg::DGArgs<double>> tp, ta, tpu, tr;
  for (int j = 0; j < np; ++j) {
    hpmg_ctx* h = hs[j];
    DGLevel& L = h->dg[0];
    hpmg::DGArgs<double> a = dg_args<double>(h, L);
    a.u_in = B->p + off0[j];
    a.tr_out = L.d.tr[0];
    add_dg_items(tp, a, L.N, R);
    hpmg::DGArgs<double> c = dg_args<double>(h, L);
    c.u_in = B->p + off0[j];
    c.tr_in = L.d.tr[0];
    c.out = B->q + off0[j];
    add_dg_items(ta, c, L.N, R);
    hpmg::DGArgs<double> pu = dg_args<double>(h, L);
    pu.tr_out = L.d.tr[0];
    add_dg_items(tpu, pu, L.N, R);
    hpmg::DGArgs<double> rr = dg_args<double>(h, L);
    rr.tr_in = L.d.tr[0];
    add_dg_items(tr, rr, L.N, R);
  }
  B->applyp.push_back(bld.dg<double>(hpmg::BOP_PROJECT, tp));
  B->applyp.push_back(bld.dg<double>(hpmg::BOP_APPLY, ta));
  // the residual launches share one argument table whose u, b are the
  // caller's, set per call: [0, np) projection of u, [np, 2np) b - A u
  // into r, [2np, 3np) the same into z (the true-residual check, which must
  // leave q, read by the next iteration, intact)
  std::vector<hpmg::DGArgs<double>> all = tpu.args;
  for (int k = 1; k <= 2; ++k)
    for (int j = 0; j < np; ++j) {
      all.push_back(tr.args[j]);
      all.back().out = (k == 1 ? B->r : B->z) + off0[j];
    }
  B->resid_args = (hpmg::DGArgs<double>*)M.alloc(all.size() * sizeof(hpmg::DGArgs<double>));
  B->resid_args_h = all;
  auto shifted = [&](const std::vector<hpmg::WorkItem>& items, int by) {
    std::vector<hpmg::WorkItem> v = items;
    for (auto& w : v) w.x += by;
    return v;
  };
  B->proj_u = dg_launch(M, 1, hpmg::BOP_PROJECT, B->resid_args, tpu.items, tpu.items1, s);
  B->resid_r = dg_launch(M, 1, hpmg::BOP_RESID, B->resid_args, shifted(tr.items, np), shifted(tr.items1, np), s);
  B->resid_z =
      dg_launch(M, 1, hpmg::BOP_RESID, B->resid_args, shifted(tr.items, 2 * np), shifted(tr.items1, 2 * np), s);
  HIPCHK(hipStreamSynchronize(s));
  return B;
}

// Autotuner over the launch configuration (grid, split, tile): first the
// fastest (grid, split) among the candidates with tile variant 0, then,
// degree by degree, tile variant 1 for that degree's one-degree launches
// where it is faster.  Timed with events on s; work(grid, split, tile,
// reps) enqueues the timed work; `degrees` are the degrees N present.
template <class F>
void tune(const std::vector<int>& grids, const std::vector<int>& degrees, F work, hipStream_t s, int& grid,
          bool& split, int& tile) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // best of three timings of two repetitions after a warm-up: one timing
  // alone varies by a few per cent from run to run, as much as the
  // differences between the configurations
  auto timed = [&](int g, bool sp, int tl) {
    work(g, sp, tl, 1);  // warm-up
    double best = 1e30;
    for (int k = 0; k < 3; ++k) {
      HIPCHK(hipEventRecord(e0, s));
      work(g, sp, tl, 2);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, (double)ms);
    }
    return best;
  };
  double tbest = 1e30;
  tile = 0;
  for (bool sp : {true, false})
    for (int g : grids) {
      const double ms = timed(g, sp, 0);
      if (ms < tbest) {
        tbest = ms;
        grid = g;
        split = sp;
      }
    }
  for (int N : degrees) {
    const int t1 = tile | (1 << N);
    const double ms = timed(grid, true, t1);
    if (ms < tbest) {
      tbest = ms;
      tile = t1;
      split = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Degrees N of the DG launches in v.
std::vector<int> degrees_of(const std::vector<Launch>& v) {
  int mask = 0;
  for (const Launch& L : v)
    for (const int3& r : L.runs) mask |= 1 << r.x;
  std::vector<int> out;
  for (int N = 0; N < 31; ++N)
    if ((mask >> N) & 1) out.push_back(N);
  return out;
}

// Grid cap above every work list: one workgroup per item (the one-degree
// launches then take their loop-free kernels).
constexpr int kOnePerItem = 1 << 30;

// Persistent grid size (or one workgroup per item), degree split and tile variants of the V-cycle
// launches, tuned on the V-cycle of the batch (run on the current r32).
void autotune_vcycle(BatchPlan* B, hipStream_t s) {
  int grid = 1024, tile = 0;
  bool split = true;
  tune({256, 512, 1024, 2048, 4096, kOnePerItem}, degrees_of(B->vcycle),
       [&](int g, bool sp, int tl, int reps) {
         for (int i = 0; i < reps; ++i) run_grid(B->vcycle, g, sp, tl, s);
       },
       s, grid, split, tile);
  B->grid = grid;
  B->split = split;
  B->tile = tile;
}

template <typename T>
T* ws_u(BatchPlan* B);
template <>
double* ws_u<double>(BatchPlan* B) { return B->z; }
template <>
float* ws_u<float>(BatchPlan* B) { return B->z32; }
template <typename T>
T* ws_b(BatchPlan* B);
template <>
double* ws_b<double>(BatchPlan* B) { return B->r; }
template <>
float* ws_b<float>(BatchPlan* B) { return B->r32; }

// Point the staged smoothing table at u, b and copy it to the device on s.
template <typename T>
void stage_smooth(BatchPlan* B, BatchPlan::Smooth& S, int np, T* const* u, const T* const* b, hipStream_t s) {
  HIPCHK(hipEventSynchronize(S.copied));  // the previous copy has left the staging buffer
  hpmg::DGArgs<T>* a = (hpmg::DGArgs<T>*)S.host;
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < np; ++j) {
      a[k * np + j].u_in = u[j];
      a[k * np + j].u_out = u[j];
      a[k * np + j].b = b[j];
    }
  HIPCHK(hipMemcpyAsync(S.args, S.host, S.bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(S.copied, s));
}

template <typename T>
void smooth_launches(BatchPlan::Smooth& S, int nsweeps, int grid, bool split, int tile, hipStream_t s) {
  std::vector<Launch> v = {S.proj};
  for (int i = 0; i < nsweeps; ++i) v.push_back((i & 1) ? S.odd : S.even);
  run_grid(v, grid, split, tile, s);
}

// Tables of hpmg_batch_smooth for dtype T; the persistent grid is tuned on
// the workspace vectors (zeroed), never on the caller's.
template <typename T>
void prepare_smooth(BatchPlan* B, const std::vector<hpmg_handle>& hs, hipStream_t s) {
  BatchPlan::Smooth& S = B->sm[sizeof(T) == 8 ? 1 : 0];
  if (S.args) return;
  const int np = (int)hs.size(), R = B->nrhs;
  Table<hpmg::DGArgs<T>> t;
  std::vector<hpmg::DGArgs<T>> all(3 * np);
  for (int j = 0; j < np; ++j) {
    hpmg_ctx* h = hs[j];
    DGLevel& L = h->dg[0];
    DGData<T>& d = data<T>(L);
    hpmg::DGArgs<T> a = dg_args<T>(h, L);
    add_dg_items(t, a, L.N, R);
    all[j] = a;
    all[j].tr_out = d.tr[0];
    all[np + j] = a;
    all[np + j].tr_in = d.tr[0];
    all[np + j].tr_out = d.tr[1];
    all[2 * np + j] = a;
    all[2 * np + j].tr_in = d.tr[1];
    all[2 * np + j].tr_out = d.tr[0];
  }
  S.bytes = all.size() * sizeof(hpmg::DGArgs<T>);
  S.args = B->mem.alloc(S.bytes);
  HIPCHK(hipHostMalloc(&S.host, S.bytes, hipHostMallocDefault));
  std::memcpy(S.host, all.data(), S.bytes);
  HIPCHK(hipEventCreateWithFlags(&S.copied, hipEventDisableTiming));
  HIPCHK(hipEventRecord(S.copied, s));
  auto shifted = [&](const std::vector<hpmg::WorkItem>& items, int by) {
    std::vector<hpmg::WorkItem> v = items;
    for (auto& w : v) w.x += by;
    return v;
  };
  const int ni = (int)t.items.size();
  const int kind = sizeof(T) == 8 ? 1 : 0;
  S.proj = dg_launch(B->mem, kind, hpmg::BOP_PROJECT, S.args, shifted(t.items, 0), shifted(t.items1, 0), s);
  S.even = dg_launch(B->mem, kind, hpmg::BOP_SWEEP, S.args, shifted(t.items, np), shifted(t.items1, np), s);
  S.odd = dg_launch(B->mem, kind, hpmg::BOP_SWEEP, S.args, shifted(t.items, 2 * np), shifted(t.items1, 2 * np), s);
  // grid: persistent candidates and one block per item
  std::vector<T*> su(np);
  std::vector<const T*> sb(np);
  for (int j = 0; j < np; ++j) {
    su[j] = ws_u<T>(B) + B->off0[j];
    sb[j] = ws_b<T>(B) + B->off0[j];
  }
  hpmg::fill<T>(ws_u<T>(B), B->total, T(0), s);
  hpmg::fill<T>(ws_b<T>(B), B->total, T(0), s);
  stage_smooth<T>(B, S, np, su.data(), sb.data(), s);
  tune({1024, 2048, 4096, 8192, ni}, degrees_of({S.even}),
       [&](int g, bool sp, int tl, int reps) { smooth_launches<T>(S, 2 * reps, g, sp, tl, s); }, s, S.grid, S.split,
       S.tile);
}

}  // namespace

extern "C" {

hpmg_status hpmg_batch_create(const hpmg_handle* hs, int count, hpmg_batch* out) {
  try {
    require(out != nullptr, "out is NULL");
    *out = nullptr;
    require(hs != nullptr && count >= 1, "need at least one handle");
    std::unique_ptr<hpmg_batch_ctx> B(new hpmg_batch_ctx());
    for (int j = 0; j < count; ++j) {
      hpmg_ctx* h = hs[j];
      require(h != nullptr, "NULL handle in batch");
      for (int k = 0; k < j; ++k) require(hs[k] != h, "a handle appears twice in the batch");
      require(h->dim == 3, "batched solver supports dim = 3");
      require(!h->vark, "batched solver supports constant kappa");
      require(!h->adapt, "batched solver supports uniform meshes");
      require(h->p + 1 >= hpmg::BATCH_NMIN && h->p + 1 <= hpmg::BATCH_NMAX, "batched solver supports 1 <= p <= 5");
      require(h->opt.nu_pre >= 1, "batched solver needs nu_pre >= 1");
      require(h->opt.p_coarsening == 0 && h->opt.p_schedule[0] == 0 && h->opt.h_factor == 2 &&
                  h->opt.basis == 0 && h->opt.block_variant == 0 && h->opt.mfma == 0,
              "batched solver supports the default p- and h-coarsening, basis and block");
      require(h->opt.nu_pre == hs[0]->opt.nu_pre && h->opt.nu_post == hs[0]->opt.nu_post &&
                  h->opt.nu_pre_cg == hs[0]->opt.nu_pre_cg && h->opt.nu_post_cg == hs[0]->opt.nu_post_cg,
              "all problems of a batch need the same smoothing counts");
      B->hs.push_back(h);
    }
    HIPCHK(hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void**)&B->host_count, 4 * sizeof(int), hipHostMallocDefault));
    *out = B.release();
    return HPMG_OK;
  } catch (const HpmgError& e) {
    set_last_error(e.what());
    return e.st;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPMG_E_NOMEM;
  }
}

void hpmg_batch_destroy(hpmg_batch b) { delete b; }

hpmg_status hpmg_batch_tuning(hpmg_batch b, int* out) {
  if (!b || !out) {
    set_last_error("NULL argument");
    return HPMG_E_INVALID;
  }
  const BatchPlan* P = b->plan.get();
  out[0] = P ? P->grid : 0;
  out[1] = P ? (int)P->split : 0;
  for (int k = 0; k < 2; ++k) {
    out[2 + 2 * k] = P ? P->sm[k].grid : 0;
    out[3 + 2 * k] = P ? (int)P->sm[k].split : 0;
  }
  out[6] = P ? P->tile : 0;
  out[7] = P ? P->sm[0].tile : 0;
  out[8] = P ? P->sm[1].tile : 0;
  return HPMG_OK;
}

hpmg_status hpmg_batch_set_tuning(hpmg_batch b, const int* cfg) {
  try {
    require(b && cfg, "NULL argument");
    BatchPlan* P = b->plan.get();
    require(P != nullptr, "no launch plan yet: solve or smooth once first");
    const int tmask = ((1 << (hpmg::BATCH_NMAX + 1)) - 1) & ~((1 << hpmg::BATCH_NMIN) - 1);
    for (int k = 0; k < 3; ++k) {
      require(cfg[2 * k] >= 0 && (cfg[2 * k + 1] == 0 || cfg[2 * k + 1] == 1), "bad grid or split");
      require((cfg[6 + k] & ~tmask) == 0, "tile mask names a degree outside the batched range");
      require(cfg[6 + k] == 0 || cfg[2 * k + 1] == 1, "half tiles need one launch per degree");
    }
    if (cfg[0] > 0) {
      P->grid = cfg[0];
      P->split = cfg[1] != 0;
      P->tile = cfg[6];
      // the captured iteration holds the old launch configuration
      if (P->exec) (void)hipGraphExecDestroy(P->exec);
      if (P->graph) (void)hipGraphDestroy(P->graph);
      P->exec = nullptr;
      P->graph = nullptr;
    }
    for (int k = 0; k < 2; ++k)
      if (cfg[2 + 2 * k] > 0) {
        P->sm[k].grid = cfg[2 + 2 * k];
        P->sm[k].split = cfg[3 + 2 * k] != 0;
        P->sm[k].tile = cfg[7 + k];
      }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    set_last_error(e.what());
    return e.st;
  }
}

hpmg_status hpmg_batch_smooth(hpmg_batch bt, hpmg_dtype dtype, void* const* u, const void* const* b, int nsweeps,
                              int nrhs, hipStream_t stream) {
  try {
    require(bt && u && b, "NULL argument");
    require(dtype == HPMG_F64 || dtype == HPMG_F32, "bad dtype");
    require(nsweeps >= 0, "nsweeps must be >= 0");
    require(nrhs >= 1, "nrhs must be >= 1");
    const std::vector<hpmg_handle>& hs = bt->hs;
    const int np = (int)hs.size();
    for (int j = 0; j < np; ++j) {
      require(u[j] && b[j], "NULL vector in batch");
      require(hs[j]->opt.max_rhs >= nrhs, "nrhs exceeds a handle's max_rhs");
      hs[j]->trace_state[0] = hs[j]->trace_state[1] = -1;
    }
    if (!bt->plan || bt->plan->nrhs != nrhs) {
      bt->plan.reset();
      bt->plan = make_plan(hs, nrhs, bt->st);
    }
    BatchPlan* B = bt->plan.get();
    if (dtype == HPMG_F64) {
      prepare_smooth<double>(B, hs, stream);
      BatchPlan::Smooth& S = B->sm[1];
      stage_smooth<double>(B, S, np, (double* const*)u, (const double* const*)b, stream);
      smooth_launches<double>(S, nsweeps, S.grid, S.split, S.tile, stream);
    } else {
      prepare_smooth<float>(B, hs, stream);
      BatchPlan::Smooth& S = B->sm[0];
      stage_smooth<float>(B, S, np, (float* const*)u, (const float* const*)b, stream);
      smooth_launches<float>(S, nsweeps, S.grid, S.split, S.tile, stream);
    }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    set_last_error(e.what());
    return e.st;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPMG_E_NOMEM;
  }
}

hpmg_status hpmg_batch_solve(hpmg_batch bt, double* const* u, const double* const* b, int nrhs, double rtol,
                             int maxit, hpmg_solve_info* infos, hipStream_t stream) {
  try {
    require(bt && u && b, "NULL argument");
    require(nrhs >= 1, "nrhs must be >= 1");
    require(rtol > 0.0 && maxit >= 1, "bad rtol/maxit");
    const auto t0 = std::chrono::steady_clock::now();
    const std::vector<hpmg_handle>& hs = bt->hs;
    const int np = (int)hs.size(), R = nrhs;
    for (int j = 0; j < np; ++j) {
      require(u[j] && b[j], "NULL vector in batch");
      require(hs[j]->opt.max_rhs >= nrhs, "nrhs exceeds a handle's max_rhs");
      hs[j]->trace_state[0] = hs[j]->trace_state[1] = -1;
    }
    // A single segment (one problem, one right-hand side) with the FP32
    // cycle: every phase is that one problem's work, which the
    // single-problem captured iteration (the problem's own kernels, no work
    // lists or segment tables) does with less overhead.
    if (np == 1 && R == 1 && hs[0]->opt.precision == HPMG_F32)
      return hpmg_solve(hs[0], u[0], b[0], 1, rtol, maxit, infos, stream);
    hipStream_t s = bt->st;
    // work queued on the caller's stream (e.g. writes of u, b) completes first
    HIPCHK(hipStreamSynchronize(stream));
    if (!bt->plan || bt->plan->nrhs != nrhs) {
      bt->plan.reset();
      bt->plan = make_plan(hs, nrhs, s);
    }
    BatchPlan* B = bt->plan.get();
    std::vector<double*> su;
    std::vector<const double*> sb;
    for (int j = 0; j < np; ++j) {
      const size_t nd = hs[j]->ndof;
      for (int r = 0; r < R; ++r) {
        su.push_back(u[j] + r * nd);
        sb.push_back(b[j] + r * nd);
      }
      for (int k = 0; k < 3; ++k) {
        B->resid_args_h[k * np + j].u_in = u[j];
        B->resid_args_h[k * np + j].b = b[j];
      }
    }
    HIPCHK(hipMemcpyAsync(B->seg_u, su.data(), su.size() * sizeof(double*), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B->seg_b, sb.data(), sb.size() * sizeof(double*), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B->resid_args, B->resid_args_h.data(),
                          B->resid_args_h.size() * sizeof(hpmg::DGArgs<double>), hipMemcpyHostToDevice, s));
    const double rtol2 = rtol * rtol;
    int* hc = bt->host_count;
    auto sync_count = [&]() {
      HIPCHK(hipMemcpyAsync(hc, B->count, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    };
    // initial residual and its FP32 copy
    residual(B, false, s);
    hpmg::bk_dot(B->seg, B->r, B->r, nullptr, B->partial, s);
    hpmg::bk_finalize(B->seg, 4, B->partial, B->scal, rtol2, s);
    hpmg::bk_cast_down(B->seg, B->r, B->r32, B->scal, s);
    hpmg::bk_count(B->seg, B->scal, B->count, s);
    if (B->grid == 0) autotune_vcycle(B, s);
    // one flexible-CG iteration of every segment, captured once and replayed
    if (!B->exec) {
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      iteration(B, s);
      HIPCHK(hipStreamEndCapture(s, &B->graph));
      HIPCHK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    }
    sync_count();
    int it = 0;
    while (hc[0] > 0 && it < maxit) {
      HIPCHK(hipGraphLaunch(B->exec, s));
      ++it;
      sync_count();
      if (hc[1] > 0) {
        // true residual of the segments whose recurrence converged; those
        // that miss the tolerance restart from it
        residual(B, true, s);
        hpmg::bk_dot(B->seg, B->z, B->z, nullptr, B->partial, s);
        hpmg::bk_finalize(B->seg, 5, B->partial, B->scal, rtol2, s);
        hpmg::bk_select(B->seg, B->z, B->r, B->scal, s);
        hpmg::bk_cast_down(B->seg, B->r, B->r32, B->scal, s);
        hpmg::bk_count(B->seg, B->scal, B->count, s);
        sync_count();
      }
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (infos) {
      std::vector<double> sc((size_t)B->seg.nseg * hpmg::BATCH_SCAL);
      HIPCHK(hipMemcpy(sc.data(), B->scal, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int j = 0; j < np; ++j) {
        hpmg_solve_info& I = infos[j];
        I.iterations = 0;
        I.initial_residual = 0.0;
        I.final_residual = 0.0;
        for (int r = 0; r < R; ++r) {
          const double* q = &sc[(size_t)(j * R + r) * hpmg::BATCH_SCAL];
          I.iterations = std::max(I.iterations, (int)q[13]);
          I.initial_residual = std::max(I.initial_residual, std::sqrt(q[9]));
          I.final_residual = std::max(I.final_residual, std::sqrt(q[12]));
        }
        for (int k = 0; k < 256; ++k) I.residual_history[k] = 0.0;
        I.seconds = secs;
      }
    }
    if (hc[2] > 0) {
      set_last_error("breakdown (non-finite value or zero curvature) in a batched solve");
      return HPMG_E_BREAKDOWN;
    }
    if (hc[0] > 0 || hc[3] > 0) {
      set_last_error(hc[3] > 0 ? "true residual stagnates above rtol (FP64 rounding floor of b - A u)"
                               : "maximum number of iterations reached");
      return HPMG_E_NOT_CONVERGED;
    }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    set_last_error(e.what());
    return e.st;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HPMG_E_NOMEM;
  }
}

}  // extern "C"
