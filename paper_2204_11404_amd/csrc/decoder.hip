// Decoding of the memory experiment (Sec. III.B): syndromes of consecutive
// rounds are compared to find detection events, the events are paired by a
// minimum-weight perfect matching, and the logical is read from the final
// measurement of the data qubits after the recovery.  Z basis (logical |0>):
// Z checks and Z_L; X basis (logical |+>, X-basis final outcomes): the same
// construction with the X checks and X_L.
//
// Host code (no kernels).  Included by qecsv.hip after the layout builder.
//
// Graph (Z basis; the X basis swaps the check type): one node per (Z check,
// layer), layers 0..R-1 for the rounds and R for the Z checks recomputed
// from the final data bits, plus one boundary
// node.  A data qubit in two Z checks joins them within a layer, a data qubit
// in one Z check joins it to the boundary, consecutive layers of a check are
// joined (measurement errors).  The checks of a round are measured one after
// another with the single ancilla (Sec. II.B): an X error on a data qubit
// shared by checks A (measured first) and B between their measurements in
// round r flips B in layer r and A in layer r + 1, so that qubit also joins
// (B, r) and (A, r + 1).  Every edge has weight 1 and flips the logical parity
// iff its data qubit lies on Z_L = Z_1 ... Z_d (the top row).
//
// Matching: exact, by dynamic programming over subsets of the events (the
// lowest unmatched event goes to the boundary or to another event).  Besides
// the minimum weight, the set of logical parities reachable at that weight is
// kept (path parities of all shortest paths, all minimum matchings), so a
// trajectory whose minimum-weight corrections disagree on the logical is
// reported as ambiguous; its failed flag then follows the first minimum found
// in a fixed order (boundary before pairs, lower partner first).

namespace {

constexpr int kDecodeMaxEvents = 22;

struct ZGraph {
  int d = 0, R = 0, nz = 0;
  int nodes = 0;  // nz * (R + 1) + 1; boundary = nodes - 1
  std::vector<std::vector<int>> zsup;  // data labels of each Z check
  std::vector<int> zidx;               // template index of each Z check
  std::vector<uint8_t> r0;             // trivial raw bit of each Z check
  std::vector<int> dist;               // [nodes][nodes]
  std::vector<uint8_t> par;            // [nodes][nodes] parity set: bit v = parity v reachable
  int basis = 1;                       // type of the decoded checks (1 = Z)
  bool on_logical(int label) const { return basis == 1 ? label <= d : (label - 1) % d == 0; }
};

// Builds the graph and all-pairs shortest-path lengths and parity sets (BFS:
// unit weights, the parity set of a node at distance k is the union over its
// neighbours at distance k - 1 of their sets shifted by the edge's flip set).
// basis 1: Z checks and Z_L = Z_1 ... Z_d (top row); basis 0: X checks and
// X_L on the first column (labels 1, d + 1, ...), for the X-basis memory.
ZGraph make_zgraph(int d, int rounds, int gateset, int basis) {
  ZGraph g;
  g.d = d;
  g.R = rounds;
  g.basis = basis;
  const std::vector<Stab> st = code_layout(d);
  for (int i = 0; i < (int)st.size(); ++i) {
    if (st[i].type != basis) continue;
    std::vector<int> sup;
    for (int q : st[i].slot)
      if (q) sup.push_back(q);
    g.zidx.push_back(i);
    g.r0.push_back(gateset == SV_GATESET_CR ? (uint8_t)((sup.size() / 2) % 2) : 0);
    g.zsup.push_back(sup);
  }
  g.nz = (int)g.zsup.size();
  g.nodes = g.nz * (rounds + 1) + 1;
  const int B = g.nodes - 1;
  // adjacency with flip sets (bit 0: even, bit 1: odd), parallel edges merged
  std::vector<std::map<int, uint8_t>> adj(g.nodes);
  auto add = [&](int a, int b, int flip) {
    const uint8_t f = (uint8_t)(1u << flip);
    adj[a][b] |= f;
    adj[b][a] |= f;
  };
  std::map<int, std::vector<int>> owners;
  for (int k = 0; k < g.nz; ++k)
    for (int q : g.zsup[k]) owners[q].push_back(k);
  for (int r = 0; r <= rounds; ++r) {
    for (const auto& kv : owners) {
      const int flip = g.on_logical(kv.first) ? 1 : 0;
      if (kv.second.size() == 2) {
        add(kv.second[0] + g.nz * r, kv.second[1] + g.nz * r, flip);
        // owners are listed in measurement order
        if (r < rounds) add(kv.second[0] + g.nz * (r + 1), kv.second[1] + g.nz * r, flip);
      } else {
        add(kv.second[0] + g.nz * r, B, flip);
      }
    }
    if (r < rounds)
      for (int k = 0; k < g.nz; ++k) add(k + g.nz * r, k + g.nz * (r + 1), 0);
  }
  g.dist.assign((size_t)g.nodes * g.nodes, -1);
  g.par.assign((size_t)g.nodes * g.nodes, 0);
  for (int s = 0; s < g.nodes; ++s) {
    int* D = &g.dist[(size_t)s * g.nodes];
    uint8_t* P = &g.par[(size_t)s * g.nodes];
    std::vector<int> frontier{s};
    D[s] = 0;
    P[s] = 1;
    while (!frontier.empty()) {
      std::vector<int> next;
      for (int u : frontier)
        for (const auto& e : adj[u]) {
          const int v = e.first;
          if (D[v] >= 0 && D[v] != D[u] + 1) continue;
          if (D[v] < 0) {
            D[v] = D[u] + 1;
            next.push_back(v);
          }
          uint8_t sh = 0;  // P[u] shifted by every flip in the edge's set
          if (e.second & 1) sh |= P[u];
          if (e.second & 2) sh |= (uint8_t)(((P[u] & 1) << 1) | ((P[u] >> 1) & 1));
          P[v] |= sh;
        }
      frontier.swap(next);
    }
  }
  return g;
}

uint8_t xor_sets(uint8_t a, uint8_t b) {
  uint8_t r = 0;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      if (((a >> x) & 1) && ((b >> y) & 1)) r |= (uint8_t)(1u << (x ^ y));
  return r;
}

struct DecodeOut {
  int weight = 0;
  uint8_t failed = 0, ambiguous = 0, ok = 1;
};

// One trajectory: records [R][n_stab] raw bits, final data bits [d*d].
DecodeOut decode_one(const ZGraph& g, int n_stab, const uint8_t* rec, const uint8_t* bits,
                     std::vector<int>& cost, std::vector<uint8_t>& pset, std::vector<uint8_t>& cano) {
  DecodeOut out;
  std::vector<uint8_t> prev(g.nz, 0);
  std::vector<int> ev;
  for (int r = 0; r <= g.R; ++r)
    for (int k = 0; k < g.nz; ++k) {
      uint8_t s;
      if (r < g.R) {
        s = rec[(size_t)r * n_stab + g.zidx[k]] ^ g.r0[k];
      } else {
        s = 0;
        for (int q : g.zsup[k]) s ^= bits[q - 1];
      }
      if (s ^ prev[k]) ev.push_back(k + g.nz * r);
      prev[k] = s;
    }
  int raw = 0;
  for (int q = 1; q <= g.d * g.d; ++q)
    if (g.on_logical(q)) raw ^= bits[q - 1];
  const int ne = (int)ev.size();
  if (ne > kDecodeMaxEvents) {
    out.ok = 0;
    return out;
  }
  const int B = g.nodes - 1;
  const size_t full = (size_t)1 << ne;
  cost.assign(full, INT32_MAX);
  pset.assign(full, 0);
  cano.assign(full, 0);
  cost[0] = 0;
  pset[0] = 1;
  cano[0] = 0;
  for (size_t m = 1; m < full; ++m) {
    const int i = __builtin_ctzll(m);
    const int a = ev[i];
    // i to the boundary
    {
      const size_t rest = m ^ ((size_t)1 << i);
      const int c = cost[rest] + g.dist[(size_t)a * g.nodes + B];
      const uint8_t ps = xor_sets(pset[rest], g.par[(size_t)a * g.nodes + B]);
      const uint8_t pc = cano[rest] ^ (uint8_t)((g.par[(size_t)a * g.nodes + B] & 1) ? 0 : 1);
      cost[m] = c;
      pset[m] = ps;
      cano[m] = pc;
    }
    for (int j = i + 1; j < ne; ++j) {
      if (!((m >> j) & 1)) continue;
      const size_t rest = m ^ ((size_t)1 << i) ^ ((size_t)1 << j);
      const uint8_t pp = g.par[(size_t)a * g.nodes + ev[j]];
      const int c = cost[rest] + g.dist[(size_t)a * g.nodes + ev[j]];
      if (c < cost[m]) {
        cost[m] = c;
        pset[m] = xor_sets(pset[rest], pp);
        cano[m] = cano[rest] ^ (uint8_t)((pp & 1) ? 0 : 1);
      } else if (c == cost[m]) {
        pset[m] |= xor_sets(pset[rest], pp);
      }
    }
  }
  out.weight = cost[full - 1];
  out.ambiguous = pset[full - 1] == 3;
  out.failed = (uint8_t)(raw ^ cano[full - 1]);
  return out;
}

sv_status decode_memory(int basis, int d, int gateset, int rounds, int n_traj, const uint8_t* records,
                        const uint8_t* final_bits, uint8_t* failed, uint8_t* ambiguous, int* weight) {
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  if (rounds < 1 || n_traj < 0) return fail(SV_EINVAL, "bad rounds / n_traj");
  if (n_traj > 0 && (!records || !final_bits || !failed)) return fail(SV_EINVAL, "NULL buffer");
  const ZGraph g = make_zgraph(d, rounds, gateset, basis);
  const int n_stab = d * d - 1, n = d * d;
  std::atomic<int> next{0}, overflow{0};
  auto work = [&] {
    std::vector<int> cost;
    std::vector<uint8_t> pset, cano;
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= n_traj) break;
      const DecodeOut o = decode_one(g, n_stab, records + (size_t)t * rounds * n_stab,
                                     final_bits + (size_t)t * n, cost, pset, cano);
      if (!o.ok) overflow.fetch_add(1);
      failed[t] = o.ok ? o.failed : 2;
      if (ambiguous) ambiguous[t] = o.ambiguous;
      if (weight) weight[t] = o.ok ? o.weight : -1;
    }
  };
  const int nth = std::max(1, std::min({16, (int)std::thread::hardware_concurrency(), n_traj}));
  std::vector<std::thread> pool;
  for (int i = 1; i < nth; ++i) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  if (overflow.load()) return fail(SV_ENUMERIC, "%d trajectories with more than %d detection events", overflow.load(),
                                   kDecodeMaxEvents);
  return SV_OK;
}

}  // namespace

extern "C" {

sv_status sv_decode_z(int d, int gateset, int rounds, int n_traj, const uint8_t* records,
                      const uint8_t* final_bits, uint8_t* failed, uint8_t* ambiguous, int* weight) {
  return decode_memory(1, d, gateset, rounds, n_traj, records, final_bits, failed, ambiguous, weight);
}

sv_status sv_decode_x(int d, int gateset, int rounds, int n_traj, const uint8_t* records,
                      const uint8_t* final_bits, uint8_t* failed, uint8_t* ambiguous, int* weight) {
  return decode_memory(0, d, gateset, rounds, n_traj, records, final_bits, failed, ambiguous, weight);
}

}  // extern "C"
