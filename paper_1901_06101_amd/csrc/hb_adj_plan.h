// Host-side plan of the frozen-pivot adjoint: validates the recorded
// structure, lays out one arena of doubles for every replayed factor,
// saved intermediate and cotangent, and lists the task launches.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "hb_adj.h"

// One leaf of the recorded forward run.
struct AdjLeafIn {
  int64_t row0, col0;   // first row / column in the problem
  int32_t m0, n0;
  int32_t nrec;         // iteration records (the last may have d_k = 0)
  int32_t rank_leaf;    // rank kept by the SVD re-compression
  const int32_t* rec;   // nrec records of fz_stride ints
};

struct AdjPlanIn {
  int64_t m = 0, n = 0;
  int L = 0;
  int dim = 0, dmax = 0, fz_stride = 0;
  std::vector<AdjLeafIn> leaves;              // 4^L leaves, b = t 2^L + v
  std::vector<std::vector<int>> hrank, vrank;  // per level 1..L, as the forward run merged
  // a merge whose P side holds at least 2 max(chunk_rows, k) rows runs as
  // G = min(max_chunks, rows / max(chunk_rows, k)) row chunks
  int64_t chunk_rows = 512;
  int max_chunks = 32;
};

struct AdjPhase {
  int kind, base, count;
};

struct AdjPlan {
  std::vector<AdjLeaf> leaves;
  std::vector<AdjBlock> blocks;
  std::vector<AdjMerge> merges;
  std::vector<AdjChunk> chunks;
  std::vector<int32_t> fz;
  std::vector<int32_t> tasks;          // merge / chunk ids of the merge launches
  std::vector<AdjPhase> fwd_phases;    // merge launches, forward order
  std::vector<AdjPhase> bwd_phases;    // merge launches, reverse order
  int root = 0, nb = 1;
  int64_t arena = 0;     // doubles, workspace included
  int64_t ws_off = 0;    // start of the phase workspace in the arena
  int64_t ws_size = 0;
};

// 0 on success; -1 for a record or rank list that does not describe a
// forward run of this shape.
inline int adj_plan(const AdjPlanIn& in, AdjPlan& P) {
  P = AdjPlan();
  if (in.L < 0 || in.L > 20 || in.dim < 1 || in.dim > HBA_MAXDIM) return -1;
  if (in.dmax < 1 || in.dmax > HBA_DMAX || in.fz_stride < 3 + 3 * in.dmax) return -1;
  if (in.chunk_rows < 1 || in.max_chunks < 1) return -1;
  const int nb = 1 << in.L;
  const int dm = in.dmax;
  P.nb = nb;
  if ((int64_t)in.leaves.size() != (int64_t)nb * nb) return -1;
  if ((int)in.hrank.size() != in.L || (int)in.vrank.size() != in.L) return -1;
  int64_t top = 0;
  auto take = [&](int64_t n) {
    const int64_t o = top;
    top += (std::max<int64_t>(n, 1) + 31) & ~(int64_t)31;
    return o;
  };
  const int stride = 3 + 3 * dm;
  // ---- leaves
  for (int li = 0; li < nb * nb; ++li) {
    const AdjLeafIn& f = in.leaves[li];
    const int t = li / nb, v = li % nb;
    if (f.m0 < 1 || f.n0 < 1 || f.nrec < 0 || (f.nrec > 0 && !f.rec)) return -1;
    if (t > 0 && f.n0 != in.leaves[v].n0) return -1;
    if (v > 0 && f.m0 != in.leaves[t * nb].m0) return -1;
    AdjLeaf L{};
    L.row0 = f.row0;
    L.col0 = f.col0;
    L.m0 = f.m0;
    L.n0 = f.n0;
    L.fz_off = (int32_t)(P.fz.size() / stride);
    int rb = 0, it = 0;
    for (int k = 0; k < f.nrec; ++k) {
      const int32_t* r = f.rec + (int64_t)k * in.fz_stride;
      const int nI = r[0], nJ = r[1], dk = r[2];
      if (dk == 0) {
        if (k != f.nrec - 1) return -1;
        break;
      }
      if (nI < 1 || nJ < 1 || nI > dm || nJ > dm || dk < 1 || dk > std::min(nI, nJ)) return -1;
      std::vector<char> seen_i(f.m0, 0), seen_j(f.n0, 0), seen_q(nJ, 0);
      for (int c = 0; c < nI; ++c) {
        const int i = r[3 + c];
        if (i < 0 || i >= f.m0 || seen_i[i]) return -1;
        seen_i[i] = 1;
      }
      for (int b = 0; b < nJ; ++b) {
        const int j = r[3 + in.dmax + b];
        if (j < 0 || j >= f.n0 || seen_j[j]) return -1;
        seen_j[j] = 1;
      }
      for (int q = 0; q < dk; ++q) {
        const int b = r[3 + 2 * in.dmax + q];
        if (b < 0 || b >= nJ || seen_q[b]) return -1;
        seen_q[b] = 1;
      }
      // copy with this plan's stride, unused slots zero
      std::vector<int32_t> rr(stride, 0);
      rr[0] = nI;
      rr[1] = nJ;
      rr[2] = dk;
      for (int c = 0; c < nI; ++c) rr[3 + c] = r[3 + c];
      for (int b = 0; b < nJ; ++b) rr[3 + dm + b] = r[3 + in.dmax + b];
      for (int q = 0; q < dk; ++q) rr[3 + 2 * dm + q] = r[3 + 2 * in.dmax + q];
      P.fz.insert(P.fz.end(), rr.begin(), rr.end());
      rb += dk;
      ++it;
    }
    if (rb > std::min(f.m0, f.n0) || f.rank_leaf < 0 || f.rank_leaf > rb) return -1;
    L.iters = it;
    L.rb = rb;
    L.rho = f.rank_leaf;
    L.U = take((int64_t)f.m0 * rb);
    L.Vt = take((int64_t)f.n0 * rb);
    L.it_sz = (((int64_t)f.m0 * dm + (int64_t)dm * f.n0 + 2 * dm * dm) + 31) & ~(int64_t)31;
    L.it = take(L.it_sz * it);
    L.Ub = take((int64_t)f.m0 * rb);
    L.Vb = take((int64_t)f.n0 * rb);
    L.S = take(rb);
    L.gU = take((int64_t)f.m0 * rb);
    L.gVt = take((int64_t)f.n0 * rb);
    L.gx = take((int64_t)f.m0 * in.dim);
    L.gy = take((int64_t)f.n0 * in.dim);
    L.gh = take(1);
    P.leaves.push_back(L);
    AdjBlock B{};
    B.m = f.m0;
    B.n = f.n0;
    B.r = f.rank_leaf;
    B.U = L.Ub;
    B.ldU = f.m0;
    B.Vt = L.Vb;
    B.ldVt = f.n0;
    B.S = L.S;
    B.gU = take((int64_t)f.m0 * B.r);
    B.gVt = take((int64_t)f.n0 * B.r);
    B.gS = take(B.r);
    P.blocks.push_back(B);
  }
  {
    int64_t rows = 0, cols = 0;
    for (int t = 0; t < nb; ++t) {
      if (in.leaves[t * nb].row0 != rows) return -1;
      rows += in.leaves[t * nb].m0;
    }
    for (int v = 0; v < nb; ++v) {
      if (in.leaves[v].col0 != cols) return -1;
      cols += in.leaves[v].n0;
    }
    if (rows != in.m || cols != in.n) return -1;
  }
  // ---- merges, level by level (horizontal, then vertical)
  auto phase = [&](int kind, const std::vector<int>& ids) {
    AdjPhase ph{kind, (int)P.tasks.size(), (int)ids.size()};
    P.tasks.insert(P.tasks.end(), ids.begin(), ids.end());
    return ph;
  };
  std::vector<std::vector<AdjPhase>> bwd_by_step;
  std::vector<int> cur(nb * nb);
  for (int i = 0; i < nb * nb; ++i) cur[i] = i;
  for (int l = 1; l <= in.L; ++l) {
    const int nbc = 1 << (in.L - l + 1), nbp = nbc / 2;
    const std::vector<int>& hr = in.hrank[l - 1];
    const std::vector<int>& vr = in.vrank[l - 1];
    if ((int64_t)hr.size() != (int64_t)nbc * nbp || (int64_t)vr.size() != (int64_t)nbp * nbp)
      return -1;
    for (int pass = 0; pass < 2; ++pass) {
      const int horiz = pass == 0;
      std::vector<int> nxt;
      const int base = (int)P.merges.size();
      const int ni = horiz ? nbc : nbp;
      for (int ti = 0; ti < ni; ++ti)
        for (int v = 0; v < nbp; ++v) {
          AdjMerge M{};
          M.horiz = horiz;
          if (horiz) {
            M.b1 = cur[ti * nbc + 2 * v];
            M.b2 = cur[ti * nbc + 2 * v + 1];
          } else {
            M.b1 = cur[(2 * ti) * nbp + v];
            M.b2 = cur[(2 * ti + 1) * nbp + v];
          }
          const AdjBlock b1 = P.blocks[M.b1], b2 = P.blocks[M.b2];
          M.rows = horiz ? b1.m : b1.n;
          if ((horiz ? b2.m : b2.n) != M.rows) return -1;
          M.n1 = horiz ? b1.n : b1.m;
          M.n2 = horiz ? b2.n : b2.m;
          M.k = b1.r + b2.r;
          M.p = (int32_t)std::min<int64_t>(M.rows, M.k);
          M.rho = horiz ? hr[ti * nbp + v] : vr[ti * nbp + v];
          if (M.rho < 0 || M.rho > M.p) return -1;
          M.Ub = take(M.rows * M.p);
          M.Y = take((int64_t)M.k * M.p);
          M.S = take(M.p);
          const int64_t on = take((M.n1 + M.n2) * M.rho);
          AdjBlock O{};
          O.r = M.rho;
          O.S = M.S;
          if (horiz) {
            O.m = M.rows;
            O.n = M.n1 + M.n2;
            O.U = M.Ub;
            O.ldU = M.rows;
            O.Vt = on;
            O.ldVt = M.n1 + M.n2;
          } else {
            O.m = M.n1 + M.n2;
            O.n = M.rows;
            O.U = on;
            O.ldU = M.n1 + M.n2;
            O.Vt = M.Ub;
            O.ldVt = M.rows;
          }
          O.gU = take(O.m * O.r);
          O.gVt = take(O.n * O.r);
          O.gS = take(O.r);
          M.out = (int32_t)P.blocks.size();
          P.blocks.push_back(O);
          nxt.push_back(M.out);
          P.merges.push_back(M);
        }
      // split the tall merges over row chunks
      std::vector<int> whole, split, parts;
      for (int i = base; i < (int)P.merges.size(); ++i) {
        AdjMerge& M = P.merges[i];
        const int64_t unit = std::max<int64_t>(in.chunk_rows, M.k);
        const int64_t g = M.k >= 1 ? std::min<int64_t>(M.rows / unit, in.max_chunks) : 1;
        M.G = g >= 2 ? (int32_t)g : 1;
        if (M.G == 1) {
          whole.push_back(i);
          continue;
        }
        split.push_back(i);
        const int64_t k = M.k, rho = M.rho, gk = (int64_t)M.G * k;
        M.Bq = take(M.rows * k);
        M.Rs = take(gk * k);
        M.QX = take(gk * k);
        M.Xs = take(k * k);
        M.part = take(M.G * (2 * k * rho + k));
        M.Jm = take(k * rho);
        M.H = take(k * k);
        M.E2 = take(k * rho);
        for (int c = 0; c < M.G; ++c) {
          AdjChunk C{};
          C.merge = i;
          C.c = c;
          C.p0 = M.rows * c / M.G;
          C.p1 = M.rows * (c + 1) / M.G;
          C.o0 = (M.n1 + M.n2) * c / M.G;
          C.o1 = (M.n1 + M.n2) * (c + 1) / M.G;
          parts.push_back((int)P.chunks.size());
          P.chunks.push_back(C);
        }
      }
      P.fwd_phases.push_back(phase(ADJ_MERGE_FWD, whole));
      P.fwd_phases.push_back(phase(ADJ_MCH_FWD1, parts));
      P.fwd_phases.push_back(phase(ADJ_MCH_FWD2, split));
      P.fwd_phases.push_back(phase(ADJ_MCH_FWD3, parts));
      bwd_by_step.push_back({phase(ADJ_MCH_BWD1, parts), phase(ADJ_MCH_BWD2, split),
                             phase(ADJ_MCH_BWD3, parts), phase(ADJ_MCH_BWD4, split),
                             phase(ADJ_MERGE_BWD, whole)});
      cur = nxt;
    }
  }
  P.root = cur[0];
  for (auto it = bwd_by_step.rbegin(); it != bwd_by_step.rend(); ++it)
    P.bwd_phases.insert(P.bwd_phases.end(), it->begin(), it->end());
  // ---- phase workspaces (tasks of one launch get disjoint pieces)
  int64_t ws = 0, acc = 0;
  auto piece = [&](int64_t n) {
    const int64_t o = acc;
    acc += (std::max<int64_t>(n, 1) + 31) & ~(int64_t)31;
    return o;
  };
  auto close = [&]() {
    ws = std::max(ws, acc);
    acc = 0;
  };
  for (auto& L : P.leaves) L.ws_lf = piece(dm);
  close();
  for (auto& L : P.leaves) {
    const int64_t r = L.rb;
    L.ws_rf = piece(((int64_t)L.m0 + L.n0) * r + 6 * r * r + r);
  }
  close();
  std::vector<AdjPhase> all = P.fwd_phases;
  all.insert(all.end(), P.bwd_phases.begin(), P.bwd_phases.end());
  for (const AdjPhase& ph : all) {
    for (int t = ph.base; t < ph.base + ph.count; ++t) {
      const int id = P.tasks[t];
      if (ph.kind == ADJ_MCH_FWD1 || ph.kind == ADJ_MCH_BWD3) {
        AdjChunk& C = P.chunks[id];
        const AdjMerge& M = P.merges[C.merge];
        if (ph.kind == ADJ_MCH_FWD1)
          C.ws_f1 = piece(M.k);
        else
          C.ws_b3 = piece((C.p1 - C.p0) * (M.rho + M.k));
        continue;
      }
      AdjMerge& M = P.merges[id];
      const int64_t k = M.k, rho = M.rho, p = M.p;
      if (ph.kind == ADJ_MERGE_FWD)
        M.ws_f = piece(M.rows * k + 5 * p * p + M.rows + k);
      else if (ph.kind == ADJ_MERGE_BWD)
        M.ws_b = piece(k * rho + 2 * p * rho + p * p + p * k + k * rho + M.rows * (rho + k));
      else if (ph.kind == ADJ_MCH_FWD2)
        M.ws_f2 = piece(2 * k * k + (int64_t)M.G * k + k);
      else if (ph.kind == ADJ_MCH_BWD2)
        M.ws_b2 = piece(2 * k * rho + k * k);
    }
    close();
  }
  piece(2 * (int64_t)P.blocks[P.root].r);
  close();
  for (auto& L : P.leaves) {
    const int64_t r = L.rb, rho = L.rho;
    L.ws_rb = piece(2 * r * rho + 5 * r * r + ((int64_t)L.m0 + L.n0) * rho);
  }
  close();
  for (auto& L : P.leaves)
    L.ws_lb = piece(4 * (int64_t)dm * L.n0 + (int64_t)L.m0 * dm + 3 * (int64_t)dm * dm);
  close();
  P.ws_off = take(ws);
  P.ws_size = ws;
  P.arena = top;
  return 0;
}

// The launch sequence, shared by the GPU and by the host emulation used in
// tests: ex.launch(kind, first task, task count) runs the tasks of one
// launch, each on its own workgroup, after every earlier launch finished.
// Task g of a leaf or reduction launch is leaf (or cluster) g; task g of a
// merge-step launch is merge or chunk P.tasks[g].
// The forward part alone evaluates the frozen operator (root block
// P.blocks[P.root]).
template <class Ex>
inline void adj_execute_forward(Ex& ex, const AdjPlan& P) {
  const int nl = (int)P.leaves.size();
  ex.launch(ADJ_LEAF_FWD, 0, nl);
  ex.launch(ADJ_REC_FWD, 0, nl);
  for (const AdjPhase& ph : P.fwd_phases) ex.launch(ph.kind, ph.base, ph.count);
}

template <class Ex>
inline void adj_execute(Ex& ex, const AdjPlan& P, bool want_x, bool want_y, bool want_h) {
  const int nl = (int)P.leaves.size();
  adj_execute_forward(ex, P);
  ex.launch(ADJ_ROOT, 0, 1);
  for (const AdjPhase& ph : P.bwd_phases) ex.launch(ph.kind, ph.base, ph.count);
  ex.launch(ADJ_REC_BWD, 0, nl);
  ex.launch(ADJ_LEAF_BWD, 0, nl);
  if (want_x) ex.launch(ADJ_RED_ROWS, 0, P.nb);
  if (want_y) ex.launch(ADJ_RED_COLS, 0, P.nb);
  if (want_h) ex.launch(ADJ_RED_H, 0, 1);
}
