// Batched independent systems (many banded systems of different sizes in one
// launch sequence and one HIP graph).
//
// Systems that share (k, r) and a padded right-hand-side count are solved as
// ONE LR-SPIKE problem over their concatenated band, with a partition boundary
// at every system boundary.  The couplings B_j, C_j across a system boundary
// are zero in the concatenation, so their spikes vanish and the reduced
// interface system splits into independent per-system blocks: every
// per-partition kernel of the single-system path runs unchanged, each launch
// covering all systems of a group.  Partition sizes come from the descriptors
// or from the autotuner (one target partition size per group, chosen by
// timing candidates on the group itself, together with the choice between the
// matrix-core wave sweeps and the workgroup sweeps for K >= 16).
//
// Included by api.hip inside its anonymous namespace.

struct BatchSys {  // per system, device copy of the packing table
  int64_t n, band_off, rhs_off, row0;  // row0: first row in the group's concatenation
  int32_t nrhs, pad;
};
struct BatchChunk {  // 256 consecutive rows of one system
  int32_t sys, pad;
  int64_t row;  // first row of the chunk within the system
};

struct BatchGroup {
  int k, r, mb;              // half-bandwidth, rank, padded right-hand sides
  std::vector<int> sys;      // indices into the descriptor array
  std::vector<int> part_sys; // system (descriptor index) of every partition
  std::vector<int64_t> offs; // partition offsets (p + 1) of the concatenation
  int64_t N = 0;
  int64_t target = 0;        // target partition size used for p = 0 systems
  int wave = 1;              // matrix-core sweeps for K >= 16
  lrspike_plan plan = nullptr;
  double* band = nullptr;    // (2k+1) x N concatenated band
  double* rhs = nullptr;     // N x mb concatenated right-hand sides
  int64_t* offs_dev = nullptr;
  int* psys_dev = nullptr;   // partition -> system slot within the group (refinement norms per system)
  char* ws = nullptr;
  BatchSys* sys_dev = nullptr;
  BatchChunk* chunks_dev = nullptr;
  int nchunks = 0;
  size_t ws_cap = 0;         // bytes allocated at ws
};

struct BatchState {
  std::vector<lrspike_batch_desc> descs;
  std::vector<BatchGroup> groups;
  const double* bands_base = nullptr;
  int precision = LRSPIKE_FP64;
  hipGraphExec_t graph = nullptr;
  double* graph_rhs = nullptr;
  hipStream_t capture = nullptr;  // private stream the graph is captured on (the caller's may be the null stream)
  // groups run side by side: one stream per group (default priority), forked
  // from and joined back into the caller's (or the capture) stream by events,
  // so that a captured step is a graph with one branch per group
  std::vector<hipStream_t> gstreams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
};


// gband[(d+k) N + row0 + i] = A_s[i, i+d] (zero where i + d leaves system s)
__global__ void pack_band_kernel(const BatchSys* __restrict__ sys, const BatchChunk* __restrict__ chunks,
                                 const double* __restrict__ base, double* __restrict__ gband, int64_t N, int k) {
  const BatchChunk ch = chunks[blockIdx.x];
  const BatchSys s = sys[ch.sys];
  const int64_t i = ch.row + threadIdx.x;
  if (i >= s.n) return;
  for (int d = -k; d <= k; ++d) {
    const int64_t c = i + d;
    gband[(int64_t)(d + k) * N + s.row0 + i] =
        (c >= 0 && c < s.n) ? base[s.band_off + (int64_t)(d + k) * s.n + i] : 0.0;
  }
}

// between the per-system n_s x nrhs_s right-hand sides and the group's N x mb block
__global__ void pack_rhs_kernel(const BatchSys* __restrict__ sys, const BatchChunk* __restrict__ chunks,
                                double* __restrict__ base, double* __restrict__ g, int mb, int unpack) {
  const BatchChunk ch = chunks[blockIdx.x];
  const BatchSys s = sys[ch.sys];
  const int rows = (int)min((int64_t)256, s.n - ch.row);
  for (int o = threadIdx.x; o < rows * mb; o += blockDim.x) {
    const int i = o / mb, c = o % mb;
    const int64_t gi = (s.row0 + ch.row + i) * mb + c;
    if (unpack) {
      if (c < s.nrhs) base[s.rhs_off + (ch.row + i) * s.nrhs + c] = g[gi];
    } else {
      g[gi] = c < s.nrhs ? base[s.rhs_off + (ch.row + i) * s.nrhs + c] : 0.0;
    }
  }
}

// keep: the concatenated band, right-hand sides and workspace stay allocated
// for the next build (the autotuner's candidates share them)
static void free_group(BatchGroup& G, bool keep = false) {
  if (G.plan) {
    prof_clear(G.plan);
    free_refine_host(G.plan);
    delete G.plan;
  }
  if (!keep) {
    (void)hipFree(G.band);
    (void)hipFree(G.rhs);
    (void)hipFree(G.ws);
    G.band = G.rhs = nullptr;
    G.ws = nullptr;
    G.ws_cap = 0;
  }
  (void)hipFree(G.offs_dev);
  (void)hipFree(G.psys_dev);
  G.psys_dev = nullptr;
  (void)hipFree(G.sys_dev);
  (void)hipFree(G.chunks_dev);
  G.plan = nullptr;
  G.offs_dev = nullptr;
  G.sys_dev = nullptr;
  G.chunks_dev = nullptr;
}

// partitions of one system: the descriptor's p, or about n / target
static int sys_partitions(const lrspike_batch_desc& d, int64_t target) {
  if (d.p > 0) return d.p;
  const int K = kernel_K(d.k);
  const int64_t minrows = std::max<int64_t>(2 * (int64_t)d.k, K);
  int64_t p = (d.n + target / 2) / target;
  p = std::min<int64_t>(p, d.n / minrows);
  return (int)std::max<int64_t>(p, 1);
}

// (Re)build the group's partitioning, device tables, workspace and plan.
static int build_group(BatchState& B, BatchGroup& G, int64_t target, int wave, const lrspike_opts* opts,
                       bool keep = false) {
  free_group(G, keep);
  G.target = target;
  G.wave = wave;
  G.offs.assign(1, 0);
  G.part_sys.clear();
  std::vector<BatchSys> st;
  std::vector<BatchChunk> ch;
  std::vector<int> pslot;
  int64_t row0 = 0;
  for (size_t q = 0; q < G.sys.size(); ++q) {
    const lrspike_batch_desc& d = B.descs[G.sys[q]];
    const int p = sys_partitions(d, target);
    const int64_t base = d.n / p, extra = d.n % p;
    for (int j = 0; j < p; ++j) {
      G.offs.push_back(G.offs.back() + base + (j < extra ? 1 : 0));
      G.part_sys.push_back(G.sys[q]);
      pslot.push_back((int)q);
    }
    st.push_back({d.n, d.band_offset, d.rhs_offset, row0, d.nrhs, 0});
    for (int64_t r = 0; r < d.n; r += 256) ch.push_back({(int32_t)q, 0, r});
    row0 += d.n;
  }
  G.N = row0;
  G.nchunks = (int)ch.size();
  const int P = (int)G.part_sys.size();
  if (hipMalloc(&G.offs_dev, (P + 1) * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&G.psys_dev, P * sizeof(int)) != hipSuccess ||
      hipMalloc(&G.sys_dev, st.size() * sizeof(BatchSys)) != hipSuccess ||
      hipMalloc(&G.chunks_dev, ch.size() * sizeof(BatchChunk)) != hipSuccess ||
      (!G.band && hipMalloc(&G.band, (size_t)(2 * G.k + 1) * G.N * 8) != hipSuccess) ||
      (!G.rhs && hipMalloc(&G.rhs, (size_t)G.N * G.mb * 8) != hipSuccess))
    return LRSPIKE_ERR_HIP;
  if (hipMemcpy(G.offs_dev, G.offs.data(), (P + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.psys_dev, pslot.data(), P * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.sys_dev, st.data(), st.size() * sizeof(BatchSys), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(G.chunks_dev, ch.data(), ch.size() * sizeof(BatchChunk), hipMemcpyHostToDevice) != hipSuccess)
    return LRSPIKE_ERR_HIP;
  lrspike_plan Q = new lrspike_plan_s();
  G.plan = Q;
  make_layout(Q->L, G.N, G.k, P, G.r, prec_tsize(B.precision), G.mb, prec_refined(B.precision), 0, G.offs.data(),
              G.offs_dev, (int)G.sys.size(), G.psys_dev);
  if (G.ws_cap < Q->L.total) {
    (void)hipFree(G.ws);
    G.ws = nullptr;
    G.ws_cap = 0;
    if (hipMalloc(&G.ws, Q->L.total) != hipSuccess) return LRSPIKE_ERR_HIP;
    G.ws_cap = Q->L.total;
  }
  if (prec_refined(B.precision) && alloc_refine_host(Q)) return LRSPIKE_ERR_HIP;
  Q->precision = B.precision;
  Q->max_refine = opts->max_refine > 0 ? opts->max_refine : 30;
  Q->refine_tol = opts->refine_tol > 0 ? opts->refine_tol : 1e-13;
  Q->stream = reinterpret_cast<hipStream_t>(opts->stream);
  Q->bands = G.band;
  Q->ws = G.ws;
  Q->profiling = 0;
  Q->wave = wave;
  return 0;
}

static int factor_group(BatchState& B, BatchGroup& G) {
  lrspike_plan P = G.plan;
  LRS_LAUNCH("pack_band_kernel", pack_band_kernel, dim3(G.nchunks), dim3(256), 0, G.sys_dev, G.chunks_dev,
             B.bands_base, G.band, G.N, G.k);
  LRS_LAUNCH("state_init_kernel", state_init_kernel, dim3(1), dim3(64), 0, reinterpret_cast<int*>(P->ws + P->L.latch));
  factor_fn f = factor_for(B.precision, P->L.K);
  return f ? f(P) : LRSPIKE_ERR_NOT_SUPPORTED;
}

static int solve_group(BatchState& B, BatchGroup& G, double* rhs_base) {
  lrspike_plan P = G.plan;
  LRS_LAUNCH("pack_rhs_kernel", pack_rhs_kernel, dim3(G.nchunks), dim3(256), 0, G.sys_dev, G.chunks_dev, rhs_base,
             G.rhs, G.mb, 0);
  apply_fn f = apply_for(B.precision, P->L.K);
  if (!f) return LRSPIKE_ERR_NOT_SUPPORTED;
  int rc = f(P, G.rhs, G.mb, 0);
  if (rc) return rc;
  LRS_LAUNCH("unpack_rhs_kernel", pack_rhs_kernel, dim3(G.nchunks), dim3(256), 0, G.sys_dev, G.chunks_dev, rhs_base,
             G.rhs, G.mb, 1);
  return 0;
}

// Autotuner: for every group, time factor + solve (zero right-hand sides,
// HIP events on the plan's stream) for each candidate partition size and
// sweep kind, and keep the fastest.  Only groups with a p = 0 system tune
// the partition size.
static int autotune(BatchState& B, const lrspike_opts* opts) {
  hipStream_t st = reinterpret_cast<hipStream_t>(opts->stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LRSPIKE_ERR_HIP;
  int rc = 0;
  for (BatchGroup& G : B.groups) {
    bool tune_p = false;
    for (int s : G.sys) tune_p |= B.descs[s].p == 0;
    const int K = kernel_K(G.k);
    std::vector<int64_t> targets = tune_p ? std::vector<int64_t>{512, 1024, 2048, 4096, 8192}
                                          : std::vector<int64_t>{4096};
    std::vector<int> waves = K >= 16 ? std::vector<int>{1, 0} : std::vector<int>{1};
    float best = 1e30f;
    int64_t bt = targets[0];
    int bw = waves[0];
    for (int64_t t : targets) {
      if (t < std::max(2 * G.k, K)) continue;
      for (int w : waves) {
        if ((rc = build_group(B, G, t, w, opts, true))) break;
        if (hipMemsetAsync(G.rhs, 0, (size_t)G.N * G.mb * 8, st) != hipSuccess) { rc = LRSPIKE_ERR_HIP; break; }
        float ms = 0.f;
        for (int rep = 0; rep < 2 && !rc; ++rep) {  // the first repetition warms up
          if (hipEventRecord(e0, st) != hipSuccess) { rc = LRSPIKE_ERR_HIP; break; }
          if ((rc = factor_group(B, G))) break;
          apply_fn f = apply_for(B.precision, K);
          if (!f) { rc = LRSPIKE_ERR_NOT_SUPPORTED; break; }
          if ((rc = f(G.plan, G.rhs, G.mb, 0))) break;
          if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = LRSPIKE_ERR_HIP;
        }
        if (rc) break;
        if (ms < best) {
          best = ms;
          bt = t;
          bw = w;
        }
      }
      if (rc) break;
    }
    if (!rc) rc = build_group(B, G, bt, bw, opts);
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Streams and events of the side-by-side groups (created once per plan).
static int batch_streams(BatchState& B) {
  if (!B.fork && hipEventCreateWithFlags(&B.fork, hipEventDisableTiming) != hipSuccess) {
    B.fork = nullptr;
    return LRSPIKE_ERR_HIP;
  }
  while (B.gstreams.size() < B.groups.size()) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return LRSPIKE_ERR_HIP;
    B.gstreams.push_back(s);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return LRSPIKE_ERR_HIP;
    B.joins.push_back(e);
  }
  return 0;
}

// Factor and/or solve every group: each group on its own stream, forked from
// `base` and joined back into it, the group with the most band entries first.
static int run_batched_on(lrspike_plan P, hipStream_t base, double* rhs_base, bool factor, bool solve) {
  BatchState& B = *P->batch;
  int rc = batch_streams(B);
  if (rc) return rc;
  if (hipEventRecord(B.fork, base) != hipSuccess) return LRSPIKE_ERR_HIP;
  std::vector<int> order(B.groups.size());
  for (size_t g = 0; g < order.size(); ++g) order[g] = (int)g;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return B.groups[a].N * (2 * B.groups[a].k + 1) > B.groups[b].N * (2 * B.groups[b].k + 1);
  });
  for (int g : order) {
    BatchGroup& G = B.groups[g];
    hipStream_t s = B.gstreams[g];
    if (hipStreamWaitEvent(s, B.fork, 0) != hipSuccess) return LRSPIKE_ERR_HIP;
    G.plan->stream = s;
    if (factor && (rc = factor_group(B, G))) return rc;
    if (solve && (rc = solve_group(B, G, rhs_base))) return rc;
    if (hipEventRecord(B.joins[g], s) != hipSuccess) return LRSPIKE_ERR_HIP;
  }
  for (size_t g = 0; g < B.groups.size(); ++g)
    if (hipStreamWaitEvent(base, B.joins[g], 0) != hipSuccess) return LRSPIKE_ERR_HIP;
  return 0;
}

static int run_batched_eager(lrspike_plan P, double* rhs_base, bool factor, bool solve) {
  return run_batched_on(P, P->stream, rhs_base, factor, solve);
}
