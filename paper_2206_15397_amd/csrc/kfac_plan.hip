// Grouped plan: the K-factor step of many factors/layers as a fixed list of grouped
// launches.  Task tables (per-task parameter blocks plus block-offset maps) are built on
// the host against the caller's workspace and copied into its head by kfac_plan_upload;
// kfac_plan_launch only enqueues kernels, so it can be captured into a hipGraph.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>
#include "workspace.h"

using namespace kfac;

namespace {

constexpr int kMaxBranches = 4;     // the caller's stream plus three (four hardware queues)

enum Kind {
  K_EA_TILES, K_EA_FIN, K_EA_TILES_BF, K_EA_FIN_BF, K_OMEGA, K_GEMM, K_BF16, K_SKINNY, K_SKINNY_R, K_SPLIT, K_GRAM_P, K_GRAM_R, K_CHOLINV, K_TRTRI, K_TRMM, K_TRIDIAG, K_PREP,
  K_BISECT, K_SELECT, K_VEC, K_CLEAD, K_CLUSTER, K_BT, K_SIGN_P, K_SIGN_A, K_GEMM_SL
};

struct LaunchRec {
  int kind;
  size_t tasks_off, off_off, gx_off;
  int ntasks, blocks;
  bool ta, tb;
  double flops, bytes;   // algorithmic work of the launch (all tasks)
  int cfg;               // tile configuration (grouped fp32 GEMM) / kernel choice (bf16 sketch)
  int ord;               // ordinal among the tunable launches (-1: not tunable)
  int ncfg;              // number of configurations of the tunable unit
  int span;              // launches belonging to the tunable unit (a split-K reduction follows)
  bool split;            // fp32 GEMM launch with split-K tasks
  int branch;            // concurrent branch (stream) the launch belongs to
};

// Algorithmic work: flops of the operation as defined (padding and split-K excluded) and
// the bytes it must move at least (each operand read once, each result written once).
struct Work {
  double flops = 0, bytes = 0;
  void operator+=(const Work& o) { flops += o.flops; bytes += o.bytes; }
};
inline Work gemm_work(double M, double N, double K, bool extra) {
  return Work{2 * M * N * K, 4 * (M * K + K * N + M * N + (extra ? M * N : 0))};
}

// Serialises one launch: [tasks][off (ntasks+1)][gx (ntasks)], each 256-byte aligned.
struct Tables {
  std::vector<char> bytes;
  std::vector<LaunchRec> recs;
  int cur_branch = 0;    // branch of the launches being added
  size_t align(size_t n) {
    size_t o = (bytes.size() + 255) / 256 * 256;
    bytes.resize(o + n);
    return o;
  }
  template <typename T>
  void add(int kind, const std::vector<T>& tasks, const std::vector<int>& gx, const std::vector<int>& nblk,
           bool ta = false, bool tb = false, Work w = Work{}) {
    if (tasks.empty()) return;
    LaunchRec r{};
    r.kind = kind;
    r.flops = w.flops;
    r.bytes = w.bytes;
    r.cfg = 0;
    r.ord = -1;
    r.ncfg = 1;
    r.span = 1;
    r.ntasks = (int)tasks.size();
    r.ta = ta; r.tb = tb;
    r.branch = cur_branch;
    r.tasks_off = align(sizeof(T) * tasks.size());
    std::memcpy(bytes.data() + r.tasks_off, tasks.data(), sizeof(T) * tasks.size());
    r.off_off = align(sizeof(int) * (tasks.size() + 1));
    int* off = (int*)(bytes.data() + r.off_off);
    off[0] = 0;
    for (size_t i = 0; i < tasks.size(); ++i) off[i + 1] = off[i] + nblk[i];
    r.blocks = off[tasks.size()];
    r.gx_off = align(sizeof(int) * tasks.size());
    std::memcpy(bytes.data() + r.gx_off, gx.data(), sizeof(int) * tasks.size());
    if (r.blocks > 0) recs.push_back(r);
  }
};

struct FactorInfo {
  int d, r, l, l_pad, q;
  long ldt;
  bool exact, ea;
  int ea_ks;
  size_t ws_off, ws_bytes;   // EigWs region
  size_t ea_off, ea_bytes;   // EA split-K partials
  size_t sk_off, sk_bytes;   // whole-width sketch / Rayleigh-Ritz split-K partials
};

struct LayerInfo {
  size_t off, bytes;
};

}  // namespace

struct kfac_plan {
  std::vector<kfac_factor_desc> f;
  std::vector<kfac_layer_desc> lyr;
  kfac_precision prec;
  float rho = 0.95f, lam = 0.1f;
  uint64_t seed = 0;
  uint32_t inv = 0;
  int do_ea = 1, do_eig = 1, do_pre = 1;
  std::vector<FactorInfo> fi;
  std::vector<LayerInfo> li;
  size_t table_bytes = 0;      // reserved head of the workspace
  size_t ws_bytes = 0;
  Tables tab;                  // built by upload
  std::vector<int> gemm_cfg;   // tuned tile configuration per fp32 GEMM launch (-1: default)
  char* dev = nullptr;         // uploaded workspace base
  // concurrent branches: every layer (with its two factors) and every factor no layer uses
  // belongs to one branch; branch b > 0 runs on stream[b - 1], forked from and joined into
  // the caller's stream around the launch sequence
  int nbranch = 1;
  std::vector<int> fbranch, lbranch;
  hipStream_t stream[kMaxBranches - 1] = {};
  hipEvent_t fork = nullptr, join[kMaxBranches - 1] = {};
};

namespace {

// Default tile configuration of a grouped fp32 GEMM launch: the largest tile that still
// gives at least ~2 workgroups per compute unit; 96 x 128 when every task has M = 96 k.
int default_gemm_cfg(const std::vector<GemmP>& g) {
  long t64 = 0, t128 = 0, t96 = 0;
  bool m96 = true;
  for (const GemmP& q : g) {
    t64 += (long)gemm_g_blocks_x(q, 0) * gemm_g_blocks_y(q, 0);
    t128 += (long)gemm_g_blocks_x(q, 1) * gemm_g_blocks_y(q, 1);
    t96 += (long)gemm_g_blocks_x(q, 2) * gemm_g_blocks_y(q, 2);
    if (q.M % 96 != 0) m96 = false;
  }
  if (m96 && t96 >= 512) return 2;
  if (t128 >= 512) return 1;
  (void)t64;
  return 0;
}

// Adds one grouped fp32 GEMM launch, with its tuned (or default) tile configuration.
void add_gemm(kfac_plan* P, Tables& T, int& ord, const std::vector<GemmP>& g, bool ta, bool tb, Work w) {
  if (g.empty()) return;
  const int o = ord++;
  bool skinny_ok = !ta && !tb;                    // the skinny tile: no transposes, M <= 288
  for (const GemmP& q : g) skinny_ok = skinny_ok && q.M <= 288 && q.ksplit <= 1;
  int cfg = (o < (int)P->gemm_cfg.size() && P->gemm_cfg[o] >= 0) ? P->gemm_cfg[o] : default_gemm_cfg(g);
  if (cfg == kGemmConfigs - 1 && !skinny_ok) cfg = default_gemm_cfg(g);
  std::vector<int> gx, nb;
  for (const GemmP& q : g) {
    gx.push_back(gemm_g_blocks_x(q, cfg));
    nb.push_back(gemm_g_blocks_x(q, cfg) * gemm_g_blocks_y(q, cfg));
  }
  const size_t before = T.recs.size();
  T.add(K_GEMM, g, gx, nb, ta, tb, w);
  // split-K tasks: slices summed and the epilogue applied by a second launch
  std::vector<GemmP> gs;
  std::vector<int> gxs, nbs;
  for (const GemmP& q : g)
    if (q.ksplit > 1) { gs.push_back(q); gxs.push_back(gemm_slice_blocks(q)); nbs.push_back(gemm_slice_blocks(q)); }
  if (T.recs.size() > before) {
    LaunchRec& r = T.recs.back();
    r.cfg = cfg;
    r.ord = o;
    r.ncfg = skinny_ok ? kGemmConfigs : kGemmConfigs - 1;
    r.split = !gs.empty();
    r.span = gs.empty() ? 1 : 2;
  }
  if (!gs.empty()) T.add(K_GEMM_SL, gs, gxs, nbs);
}

// Task tables of branch `br` (its factors and layers) for workspace base `base` (null:
// sizes only) and status pointer, appended to T; gord numbers the tunable launches.
void build_branch(kfac_plan* P, char* base, int* status, Tables& T, int br, int& gord) {
  const bool bf = (P->prec == KFAC_SKETCH_BF16);
  const bool sp = (P->prec == KFAC_SKETCH_SPLIT);
  T.cur_branch = br;
  auto in_f = [&](size_t i) { return P->fbranch.empty() ? br == 0 : P->fbranch[i] == br; };
  // branch nbranch: the layers whose two factors sit in different branches, after the join
  auto in_l = [&](size_t l) {
    if (P->lbranch.empty()) return br == 0;
    return br == P->nbranch ? P->lbranch[l] == -1 : P->lbranch[l] == br;
  };
  const size_t head = P->table_bytes;
  auto wsp = [&](size_t off) -> void* { return base ? (void*)(base + head + off) : nullptr; };
  std::vector<EigWs> W;
  for (size_t i = 0; i < P->f.size(); ++i)
    W.emplace_back(P->fi[i].d, P->fi[i].r, P->f[i].p, (int)P->prec, wsp(P->fi[i].ws_off));

  // ---- EA --------------------------------------------------------------------------
  if (P->do_ea) {
    // fp32 activations use the fp32-MFMA kernel, bf16 activations the bf16-MFMA one
    for (int xb = 0; xb < 2; ++xb) {
      std::vector<EaTask> t, tf;
      std::vector<int> gx, nb, gxf, nbf;
      Work wt, wf;
      for (size_t i = 0; i < P->f.size(); ++i) {
        const kfac_factor_desc& F = P->f[i];
        const FactorInfo& I = P->fi[i];
        if (!in_f(i) || !I.ea || (F.xtype == KFAC_BF16) != (xb == 1)) continue;
        EaTask q = make_ea_task(F.F, I.d, F.ldf, xb ? nullptr : (const float*)F.X,
                                xb ? (const uint16_t*)F.X : nullptr, (int)F.n, (int)F.d_in, F.ldx,
                                F.append_ones, P->rho, F.scale, F.F_bf16, F.ldfb, (float*)wsp(I.ea_off), I.ea_ks);
        const int tiles = q.T * (q.T + 1) / 2;
        t.push_back(q); gx.push_back(tiles); nb.push_back((tiles * I.ea_ks + 7) / 8 * 8);   // XCD eighths
        if (I.ea_ks > 1) {
          const int fb = tiles * ea_finalize_chunks(xb == 1);
          tf.push_back(q); gxf.push_back(fb); nbf.push_back(fb);
        }
        // sums over the upper triangle; F: upper half read, full F written (+ bf16 shadow)
        const double d = I.d, n = (double)F.n;
        const Work x{n * d * (d + 1), n * (double)F.d_in * (xb ? 2 : 4)};
        const Work f{0, 4 * d * (d + 1) / 2 + 4 * d * d + (F.F_bf16 ? 2 * d * d : 0)};
        if (I.ea_ks > 1) { wt += x; wf += f; } else { wt += x; wt += f; }
      }
      T.add(xb ? K_EA_TILES_BF : K_EA_TILES, t, gx, nb, false, false, wt);
      T.add(xb ? K_EA_FIN_BF : K_EA_FIN, tf, gxf, nbf, false, false, wf);
    }
  }
  if (P->do_eig) {
    // ---- randomized range finder with CholeskyQR2 -----------------------------------
    std::vector<int> rnd;
    for (size_t i = 0; i < P->f.size(); ++i)
      if (in_f(i) && !P->fi[i].exact) rnd.push_back((int)i);
    std::vector<float*> basis(P->f.size(), nullptr), spare(P->f.size(), nullptr);
    if (!rnd.empty()) {
      std::vector<OmegaTask> om;
      std::vector<int> gx, nb;
      Work wo;
      for (int i : rnd) {
        const FactorInfo& I = P->fi[i];
        // bf16-sketch mode: the sketch reads only the bf16 copy of Omega^T
        wo += Work{0, (double)I.l * I.d * (bf ? 2 : 4)};
        OmegaTask q = make_omega_task(I.d, I.l, I.d, I.l_pad, P->seed, P->f[i].stream_id, P->inv,
                                      bf ? nullptr : W[i].OmT, I.ldt, bf ? W[i].OmTb : nullptr, nullptr, 0, nullptr);
        dim3 g = omega_grid(q);
        om.push_back(q); gx.push_back((int)g.x); nb.push_back((int)(g.x * g.y));
      }
      T.add(K_OMEGA, om, gx, nb, false, false, wo);
      for (int i : rnd) { basis[i] = W[i].Yt; spare[i] = W[i].Qt; }
      const int qmax = [&] { int m = 0; for (int i : rnd) m = std::max(m, P->fi[i].q); return m; }();
      for (int it = 0; it <= qmax; ++it) {
        // sketch (it == 0: F Omega) or power step (F Q), into the buffer that will hold
        // the new basis after CholeskyQR2
        std::vector<int> act;
        for (int i : rnd) if (it <= P->fi[i].q) act.push_back(i);
        if (act.empty()) break;
        Work ws;
        for (int i : act) {
          const double l = P->fi[i].l, d = P->fi[i].d;
          ws += bf ? Work{2 * l * d * d, 2 * d * d + 2 * l * d + 4 * l * d} : gemm_work(l, d, d, false);
        }
        if (sp) {
          // split-bf16 products of the fp32 operands (whole sketch width per workgroup)
          std::vector<SplitTask> g;
          std::vector<ReduceTask> gr;
          std::vector<int> gx2, nb2, gxr, nbr;
          for (int i : act) {
            const FactorInfo& I = P->fi[i];
            const float* A = (it == 0) ? W[i].OmT : basis[i];
            float* out = (it == 0) ? basis[i] : spare[i];
            const SplitTask q = make_split_task(I.l_pad, I.d, I.d, A, I.ldt, P->f[i].F, P->f[i].ldf, out, I.ldt,
                                                (float*)wsp(I.sk_off), split_ksplit(I.d, I.d));
            g.push_back(q); gx2.push_back(q.tiles_n); nb2.push_back(split_blocks(q));
            if (q.ksplit > 1) {
              const ReduceTask rq = make_reduce_task(q.M, q.N, q.part, q.C, q.ldc, q.ksplit);
              gr.push_back(rq); gxr.push_back(reduce_blocks(rq)); nbr.push_back(reduce_blocks(rq));
            }
          }
          T.add(K_SPLIT, g, gx2, nb2, false, false, ws);
          T.add(K_SKINNY_R, gr, gxr, nbr);
        } else if (bf) {
          // tunable unit: 0 = 96 x 128 tiles, 1 = skinny full-M tiles with split-K
          const int o = gord++;
          int dmax = 0;
          for (int i : act) dmax = std::max(dmax, P->fi[i].d);
          const int cfg = (o < (int)P->gemm_cfg.size() && P->gemm_cfg[o] >= 0) ? P->gemm_cfg[o] : (dmax >= 2048 ? 1 : 0);
          const size_t before = T.recs.size();
          if (cfg == 0) {
            std::vector<BfGemmTask> g;
            std::vector<int> gx2, nb2;
            for (int i : act) {
              const FactorInfo& I = P->fi[i];
              const uint16_t* A = (it == 0) ? W[i].OmTb : W[i].Qtb;
              float* out = (it == 0) ? basis[i] : spare[i];
              BfGemmTask q = make_bf16_task(I.l_pad, I.d, I.d, A, I.ldt, P->f[i].F_bf16, P->f[i].ldfb, out, I.ldt);
              g.push_back(q); gx2.push_back(bf16_task_blocks(q)); nb2.push_back(bf16_task_blocks(q));
            }
            T.add(K_BF16, g, gx2, nb2, false, false, ws);
          } else {
            std::vector<SkinnyTask> g;
            std::vector<ReduceTask> gr;
            std::vector<int> gx2, nb2, gxr, nbr;
            for (int i : act) {
              const FactorInfo& I = P->fi[i];
              const uint16_t* A = (it == 0) ? W[i].OmTb : W[i].Qtb;
              float* out = (it == 0) ? basis[i] : spare[i];
              SkinnyTask q = make_skinny_task(I.l_pad, I.d, I.d, A, I.ldt, P->f[i].F_bf16, P->f[i].ldfb, out, I.ldt,
                                              (float*)wsp(I.sk_off), skinny_ksplit(I.d, I.d));
              g.push_back(q); gx2.push_back(q.tiles_n); nb2.push_back(skinny_blocks(q));
              if (q.ksplit > 1) {
                const ReduceTask rq = make_reduce_task(q.M, q.N, q.part, q.C, q.ldc, q.ksplit);
                gr.push_back(rq); gxr.push_back(reduce_blocks(rq)); nbr.push_back(reduce_blocks(rq));
              }
            }
            T.add(K_SKINNY, g, gx2, nb2, false, false, ws);
            T.add(K_SKINNY_R, gr, gxr, nbr);
          }
          if (T.recs.size() > before) {
            LaunchRec& r0 = T.recs[before];
            r0.cfg = cfg;
            r0.ord = o;
            r0.ncfg = 2;
            r0.span = (int)(T.recs.size() - before);
          }
        } else {
          std::vector<GemmP> g;
          std::vector<int> gx2, nb2;
          for (int i : act) {
            const FactorInfo& I = P->fi[i];
            GemmP q{};
            q.M = I.l_pad; q.N = I.d; q.K = I.d;
            q.A = (it == 0) ? W[i].OmT : basis[i]; q.lda = I.ldt;
            q.B = P->f[i].F; q.ldb = P->f[i].ldf;
            q.C = (it == 0) ? basis[i] : spare[i]; q.ldc = I.ldt;
            q.alpha = 1.f; q.ones_col = -1;
            g.push_back(q);
          }
          add_gemm(P, T, gord, g, false, false, ws);
        }
        if (it > 0) for (int i : act) std::swap(basis[i], spare[i]);
        // CholeskyQR2 on basis[i] for the final basis (pass 0 basis -> spare, pass 1 spare ->
        // basis); inside the power iteration one pass, basis -> spare, then swapped: the
        // next product and the final two passes restore orthonormality
        auto npass_of = [&](int i) { return it < P->fi[i].q ? 1 : 2; };
        int npass_max = 1;
        for (int i : act) npass_max = std::max(npass_max, npass_of(i));
        for (int pass = 0; pass < npass_max; ++pass) {
          std::vector<GramP> gp;
          std::vector<CholInvTask> ch;
          std::vector<TrmmTask> tm;
          std::vector<int> gxg, nbg, gxr, nbr, gxc, nbc, gxt, nbt, gxi, nbi;
          Work wg, wr, wc, wi, wm;
          for (int i : act) {
            const int npass = npass_of(i);
            if (pass >= npass) continue;
            const FactorInfo& I = P->fi[i];
            const double l = I.l, d = I.d;
            wg += Work{l * (l + 1) * d, 4 * l * d};
            wr += Work{0, 8 * l * l};
            wc += Work{l * l * l / 3, 16 * l * l};       // Cholesky
            wi += Work{l * l * l / 3, 16 * l * l};       // triangular inverse
            // the bf16 copy of Q only where a bf16 power-iteration product follows (the
            // Rayleigh-Ritz product and U = QP take the fp32 basis)
            const bool qb = bf && pass == npass - 1 && it < I.q;
            wm += Work{l * (l + 1) * d, 8 * l * d + 8 * l * l / 2 + (qb ? 2 * l * d : 0)};
            float* src = pass == 0 ? basis[i] : spare[i];
            float* dst = pass == 0 ? spare[i] : basis[i];
            GramP g = make_gram_task(src, I.ldt, src, I.ldt, I.l_pad, I.d, 1, W[i].part, W[i].G, I.l_pad, status);
            const int tiles = gram_tiles(I.l_pad, 1);
            gp.push_back(g); gxg.push_back(tiles); nbg.push_back(tiles * g.ksplit);
            gxr.push_back(tiles); nbr.push_back(tiles * gram_reduce_slices());
            // the second pass may be kept out (first pass already orthonormal to 2^-24)
            int* keep = (pass == 1) ? W[i].fail + 1 : nullptr;
            CholInvTask c{W[i].G, I.l_pad, I.l, I.d, W[i].Wc, I.l_pad, I.l_pad, W[i].Li, status, W[i].fail, 0,
                          keep, kQrKeepTol};
            ch.push_back(c); gxc.push_back(1); nbc.push_back(1);
            gxi.push_back(trtri_col_blocks(I.l_pad)); nbi.push_back(trtri_col_blocks(I.l_pad));
            TrmmTask tt{W[i].Wc, I.l_pad, I.l, src, I.ldt, I.d, dst, I.ldt,
                        qb ? W[i].Qtb : nullptr, I.ldt, I.l_pad, keep};
            const int bx = trmm_blocks_x(I.d), by = trmm_blocks_y(I.l_pad);
            tm.push_back(tt); gxt.push_back(bx); nbt.push_back(bx * by);
          }
          T.add(K_GRAM_P, gp, gxg, nbg, false, false, wg);
          T.add(K_GRAM_R, gp, gxr, nbr, false, false, wr);
          T.add(K_CHOLINV, ch, gxc, nbc, false, false, wc);
          for (auto& c : ch) c.attempt = 1;
          T.add(K_CHOLINV, ch, gxc, nbc);   // re-run only where attempt 0 broke down
          T.add(K_TRTRI, ch, gxi, nbi, false, false, wi);
          T.add(K_TRMM, tm, gxt, nbt, false, false, wm);
        }
        for (int i : act)
          if (npass_of(i) == 1) std::swap(basis[i], spare[i]);   // the one-pass basis is in spare
      }
      // Rayleigh-Ritz: W = F Q into spare (fp32 tiles; split-bf16 in the bf16-sketch mode),
      // C = Q^T W (fp64) into G
      std::vector<GemmP> g;
      std::vector<SplitTask> gs;
      std::vector<ReduceTask> gsr;
      std::vector<int> gx2, nb2, gxs, nbs, gxsr, nbsr;
      std::vector<GramP> gp;
      std::vector<int> gxg, nbg, gxr, nbr;
      Work wrr, wg, wr;
      for (int i : rnd) {
        const FactorInfo& I = P->fi[i];
        const double l = I.l, d = I.d;
        wrr += gemm_work(l, d, d, false);
        wg += P->f[i].variant == KFAC_RSVD ? Work{l * (l + 1) * d, 4 * l * d} : Work{2 * l * l * d, 8 * l * d};
        wr += Work{0, 8 * l * l};
        if (bf || sp) {
          const SplitTask q = make_split_task(I.l_pad, I.d, I.d, basis[i], I.ldt, P->f[i].F, P->f[i].ldf, spare[i],
                                              I.ldt, (float*)wsp(I.sk_off), split_ksplit(I.d, I.d));
          gs.push_back(q); gxs.push_back(q.tiles_n); nbs.push_back(split_blocks(q));
          if (q.ksplit > 1) {
            const ReduceTask rq = make_reduce_task(q.M, q.N, q.part, q.C, q.ldc, q.ksplit);
            gsr.push_back(rq); gxsr.push_back(reduce_blocks(rq)); nbsr.push_back(reduce_blocks(rq));
          }
        } else {
          GemmP q{};
          q.M = I.l_pad; q.N = I.d; q.K = I.d;
          q.A = basis[i]; q.lda = I.ldt; q.B = P->f[i].F; q.ldb = P->f[i].ldf;
          q.C = spare[i]; q.ldc = I.ldt; q.alpha = 1.f; q.ones_col = -1;
          g.push_back(q);
        }
        // SREVD: C = Q^T W; RSVD: the Gram W^T W of B^T = W = F Q
        const int sv = P->f[i].variant == KFAC_RSVD ? 1 : 0;
        GramP gr = sv ? make_gram_task(spare[i], I.ldt, spare[i], I.ldt, I.l_pad, I.d, 1, W[i].part, W[i].G,
                                       I.l_pad, status)
                      : make_gram_task(basis[i], I.ldt, spare[i], I.ldt, I.l_pad, I.d, 0, W[i].part, W[i].G,
                                       I.l_pad, status);
        const int tiles = gram_tiles(I.l_pad, sv);
        gp.push_back(gr); gxg.push_back(tiles); nbg.push_back(tiles * gr.ksplit);
        gxr.push_back(tiles); nbr.push_back(tiles * gram_reduce_slices());
      }
      if (bf || sp) {
        T.add(K_SPLIT, gs, gxs, nbs, false, false, wrr);
        T.add(K_SKINNY_R, gsr, gxsr, nbsr);
      } else {
        add_gemm(P, T, gord, g, false, false, wrr);
      }
      T.add(K_GRAM_P, gp, gxg, nbg, false, false, wg);
      T.add(K_GRAM_R, gp, gxr, nbr, false, false, wr);
    }
    // ---- small eigensolver (randomized: C = Q^T F Q; exact: F itself) --------------
    std::vector<EigTask> et;
    std::vector<int> one, onen, gxb, nbb, gxv, nbv, gxbt, nbbt;
    Work wtri, wbt;
    for (size_t i = 0; i < P->f.size(); ++i) {
      if (!in_f(i)) continue;
      const FactorInfo& I = P->fi[i];
      const kfac_factor_desc& F = P->f[i];
      const double n = I.l, r = I.r;
      wtri += Work{4 * n * n * n / 3, 8 * n * n + 16 * n};   // Householder tridiagonalisation
      wbt += Work{2 * n * n * r, 8 * n * r + 4 * n * r};    // back-transformation of r vectors
      EigTask q;
      if (I.exact)
        q = make_eig_task(nullptr, 0, F.F, F.ldf, I.d, I.d, I.r, W[i].A, W[i].V, W[i].diag, W[i].off, W[i].Z,
                          W[i].scr, F.U, F.ldu, F.D, W[i].Dd, status);
      else
        q = make_eig_task(W[i].G, I.l_pad, nullptr, 0, I.l, I.l_pad, I.r, W[i].A, W[i].V, W[i].diag, W[i].off,
                          W[i].Z, W[i].scr, W[i].P, I.r, F.D, W[i].Dd, status);
      q.svd = (!I.exact && F.variant == KFAC_RSVD) ? 1 : 0;
      et.push_back(q);
      one.push_back(1); onen.push_back(1);
      gxb.push_back(tri_bisect_blocks(q.n)); nbb.push_back(tri_bisect_blocks(q.n));
      gxv.push_back(tri_vec_blocks(q.r)); nbv.push_back(tri_vec_blocks(q.r));
    }
    T.add(K_TRIDIAG, et, one, onen, false, false, wtri);
    T.add(K_PREP, et, one, onen);
    T.add(K_BISECT, et, gxb, nbb);
    T.add(K_SELECT, et, one, onen);
    T.add(K_VEC, et, gxv, nbv);
    T.add(K_CLEAD, et, one, onen);
    T.add(K_CLUSTER, et, one, onen);
    for (const EigTask& q : et) {
      gxbt.push_back(backtransform_blocks(q.r));
      nbbt.push_back(backtransform_blocks(q.r));
    }
    T.add(K_BT, et, gxbt, nbbt, false, false, wbt);
    // ---- Ritz vectors U = Q P[:, :r] --------------------------------------------------
    {
      std::vector<GemmP> g;
      std::vector<int> gx2, nb2;
      Work wu;
      for (int i : rnd) {
        const FactorInfo& I = P->fi[i];
        wu += gemm_work(I.d, I.r, I.l, false);
        GemmP q{};
        q.M = I.d; q.N = I.r; q.K = I.l;
        // SREVD: U = Q P; RSVD: U = W P Sigma^{-1} (the eigensolver scaled P)
        q.A = P->f[i].variant == KFAC_RSVD ? spare[i] : basis[i]; q.lda = I.ldt; q.B = W[i].P; q.ldb = I.r;
        q.C = P->f[i].U; q.ldc = P->f[i].ldu; q.alpha = 1.f; q.ones_col = -1;
        g.push_back(q);
      }
      add_gemm(P, T, gord, g, true, false, wu);
    }
    // ---- column signs -------------------------------------------------------------------
    {
      std::vector<SignTask> st;
      std::vector<int> gx2, nb2;
      Work wsp, wsa;
      for (size_t i = 0; i < P->f.size(); ++i) {
        if (!in_f(i)) continue;
        const FactorInfo& I = P->fi[i];
        wsp += Work{0, 4.0 * I.d * I.r};
        wsa += Work{0, 8.0 * I.d * I.r};
        SignTask s{P->f[i].U, P->f[i].ldu, I.d, I.r, W[i].sval, W[i].sidx, sign_chunks(I.d)};
        st.push_back(s);
        const int bx = (I.r + 63) / 64;
        gx2.push_back(bx); nb2.push_back(bx * sign_chunks(I.d));
      }
      T.add(K_SIGN_P, st, gx2, nb2, false, false, wsp);
      T.add(K_SIGN_A, st, gx2, nb2, false, false, wsa);
    }
  }
  // ---- damped inverse per layer -----------------------------------------------------------
  if (P->do_pre && !P->lyr.empty()) {
    std::vector<GemmP> g1, g2, g3, g4;
    std::vector<int> x1, n1, x2, n2, x3, n3, x4, n4;
    Work w1, w2, w3, w4;
    const float inv_lam = 1.0f / P->lam;
    for (size_t l = 0; l < P->lyr.size(); ++l) {
      if (!in_l(l)) continue;
      const kfac_layer_desc& L = P->lyr[l];
      const kfac_factor_desc& A = P->f[L.fa];
      const kfac_factor_desc& G = P->f[L.fg];
      const int dg = (int)G.d, da = (int)A.d, ra = (int)A.r, rg = (int)G.r;
      w1 += gemm_work(dg, ra, da, false);
      w2 += gemm_work(dg, da, ra, true);
      w3 += gemm_work(rg, da, dg, false);
      w4 += gemm_work(dg, da, rg, true);
      Bump b(wsp(P->li[l].off));
      float* T1 = b.take<float>((size_t)dg * ra);
      float* M = b.take<float>((size_t)dg * da);
      float* T2 = b.take<float>((size_t)rg * da);
      const int ks1 = precondition_ksplit(dg, da, ra);
      float* T1p = ks1 > 1 ? b.take<float>((size_t)ks1 * dg * ra) : nullptr;
      auto push = [&](std::vector<GemmP>& v, std::vector<int>& gx, std::vector<int>& nb, const GemmP& q) {
        v.push_back(q); (void)gx; (void)nb;
      };
      GemmP q{};
      q.ones_col = -1; q.alpha = 1.f; q.lam = P->lam;
      GemmP a = q;  // T1 = J U_a diag(f_a)
      a.M = dg; a.N = ra; a.K = da; a.A = L.J; a.lda = L.ldj; a.B = A.U; a.ldb = A.ldu; a.C = T1; a.ldc = ra; a.colD = A.D;
      if (ks1 > 1) { a.ksplit = ks1; a.part = T1p; }
      push(g1, x1, n1, a);
      GemmP m = q;  // M = T1 U_a^T + J / lambda
      m.M = dg; m.N = da; m.K = ra; m.A = T1; m.lda = ra; m.B = A.U; m.ldb = A.ldu; m.C = M; m.ldc = da;
      m.X = L.J; m.ldx = L.ldj; m.beta = inv_lam;
      push(g2, x2, n2, m);
      GemmP t2 = q;  // T2 = diag(f_g) U_g^T M
      t2.M = rg; t2.N = da; t2.K = dg; t2.A = G.U; t2.lda = G.ldu; t2.B = M; t2.ldb = da; t2.C = T2; t2.ldc = da;
      t2.rowD = G.D;
      push(g3, x3, n3, t2);
      GemmP sq = q;  // S = U_g T2 + M / lambda
      sq.M = dg; sq.N = da; sq.K = rg; sq.A = G.U; sq.lda = G.ldu; sq.B = T2; sq.ldb = da; sq.C = L.S; sq.ldc = L.lds;
      sq.X = M; sq.ldx = da; sq.beta = inv_lam;
      push(g4, x4, n4, sq);
    }
    add_gemm(P, T, gord, g1, false, false, w1);
    add_gemm(P, T, gord, g2, false, true, w2);
    add_gemm(P, T, gord, g3, true, false, w3);
    add_gemm(P, T, gord, g4, false, false, w4);
  }
}

// All task tables, branch after branch (each branch's launches are in stream order).
void build_tables(kfac_plan* P, char* base, int* status, Tables& T) {
  int gord = 0;                 // ordinal of the next tunable launch
  for (int b = 0; b < P->nbranch; ++b) build_branch(P, base, status, T, b, gord);
  bool post = false;
  for (int lb : P->lbranch) post = post || lb == -1;
  if (post && P->nbranch > 1) build_branch(P, base, status, T, P->nbranch, gord);
  T.cur_branch = 0;
}

// Work estimate of one factor's share of the step (EA products, sketch / power / Rayleigh-
// Ritz products): the quantity branches are balanced on.
double factor_cost(const kfac_plan* P, size_t i) {
  const kfac_factor_desc& F = P->f[i];
  const double d = (double)F.d, l = std::min<double>((double)(F.r + F.p), d);
  double c = 2.0 * d * d * l * (F.q + 2);
  if (F.X) c += (double)F.n * d * d;
  return c;
}

// Layers (with their factors) and unused factors to branches: the layers with the largest
// EA work go to branch nb - 1, the others are spread over the branches by longest-
// processing-time on factor_cost.  A branch whose EA is light starts its eigensolver
// phases (latency-bound, few workgroups each) while the heavy-EA branch still streams its
// activations, and its preconditioner overlaps the other branch's eigensolver.
void assign_branches(kfac_plan* P, int nb) {
  const size_t nf = P->f.size(), nl = P->lyr.size();
  P->fbranch.assign(nf, -1);
  P->lbranch.assign(nl, 0);
  if (nb <= 1) { P->fbranch.assign(nf, 0); return; }
  struct Unit { std::vector<int> f; int l; double cost, ea; };
  std::vector<Unit> units;
  std::vector<char> used(nf, 0);
  for (size_t l = 0; l < nl; ++l) {
    Unit u{{}, (int)l, 0.0, 0.0};
    for (int fi : {P->lyr[l].fa, P->lyr[l].fg})
      if (!used[fi]) {
        used[fi] = 1;
        u.f.push_back(fi);
        u.cost += factor_cost(P, fi);
        if (P->f[fi].X) u.ea += (double)P->f[fi].n * P->f[fi].d * P->f[fi].d;
      }
    units.push_back(u);
  }
  for (size_t i = 0; i < nf; ++i)
    if (!used[i]) {
      const double ea = P->f[i].X ? (double)P->f[i].n * P->f[i].d * P->f[i].d : 0.0;
      units.push_back(Unit{{(int)i}, -1, factor_cost(P, i), ea});
    }
  // heavy-EA units: the largest EA works that together hold at least half of the EA
  std::vector<size_t> ord(units.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return units[a].ea > units[b].ea; });
  double ea_tot = 0.0, ea_acc = 0.0;
  for (const Unit& u : units) ea_tot += u.ea;
  std::vector<int> br(units.size(), -1);
  for (size_t k : ord) {
    if (ea_tot <= 0.0 || ea_acc >= 0.5 * ea_tot) break;
    br[k] = nb - 1;
    ea_acc += units[k].ea;
  }
  // the rest by LPT over branches 0 .. nb - 2 (all branches if nothing is heavy)
  const int nlight = (ea_acc > 0.0) ? nb - 1 : nb;
  std::vector<double> load(nb, 0.0);
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return units[a].cost > units[b].cost; });
  for (size_t k : ord) {
    if (br[k] >= 0) { load[br[k]] += units[k].cost; continue; }
    int best = 0;
    for (int b = 1; b < nlight; ++b) if (load[b] < load[best]) best = b;
    br[k] = best;
    load[best] += units[k].cost;
  }
  for (size_t k = 0; k < units.size(); ++k) {
    for (int fi : units[k].f) P->fbranch[fi] = br[k];
    if (units[k].l >= 0) P->lbranch[units[k].l] = br[k];
  }
  // a factor shared with a layer of another branch stays where it was placed first; the
  // other branch then reads its (U, D) only after the join, so such layers run in branch of
  // their first factor's owner
  for (size_t l = 0; l < nl; ++l) {
    const int a = P->fbranch[P->lyr[l].fa], g = P->fbranch[P->lyr[l].fg];
    if (a != g) P->lbranch[l] = -1;   // precondition after the join (see kfac_plan_launch)
    else P->lbranch[l] = a;
  }
}

}  // namespace

extern "C" {

kfac_status kfac_plan_create(const kfac_factor_desc* factors, int nf, const kfac_layer_desc* layers, int nl,
                             kfac_precision prec, kfac_plan** out) {
  if (!out || nf < 1 || (nl > 0 && !layers) || !factors) return KFAC_EINVAL;
  if (prec != KFAC_SKETCH_FP32 && prec != KFAC_SKETCH_BF16 && prec != KFAC_SKETCH_SPLIT) return KFAC_EINVAL;
  *out = nullptr;
  for (int i = 0; i < nf; ++i) {
    const kfac_factor_desc& F = factors[i];
    if (!F.F || F.d < 1 || F.ldf < F.d || F.r < 1 || F.r > F.d || F.p < 0 || F.q < 0 || F.q > 16) return KFAC_EINVAL;
    if (!F.U || F.ldu < F.r || !F.D) return KFAC_EINVAL;
    if (F.variant != KFAC_SREVD && F.variant != KFAC_RSVD) return KFAC_EINVAL;
    if (prec == KFAC_SKETCH_BF16 && (!F.F_bf16 || F.ldfb < F.d)) return KFAC_EINVAL;
    if (F.X) {
      if (F.n < 1 || F.d != F.d_in + (F.append_ones ? 1 : 0) || F.ldx < F.d_in || !(F.scale > 0.f)) return KFAC_EINVAL;
      if (F.xtype != KFAC_FP32 && F.xtype != KFAC_BF16) return KFAC_EINVAL;
    }
    if (std::min<int64_t>(F.r + F.p, F.d) > kPlanMaxSketch) return KFAC_EUNSUPPORTED;
  }
  for (int l = 0; l < nl; ++l) {
    const kfac_layer_desc& L = layers[l];
    if (L.fa < 0 || L.fa >= nf || L.fg < 0 || L.fg >= nf || !L.J || !L.S) return KFAC_EINVAL;
    if (L.ldj < factors[L.fa].d || L.lds < factors[L.fa].d || (const void*)L.J == (const void*)L.S) return KFAC_EINVAL;
  }
  kfac_plan* P = new (std::nothrow) kfac_plan();
  if (!P) return KFAC_EINVAL;
  P->f.assign(factors, factors + nf);
  if (nl > 0) P->lyr.assign(layers, layers + nl);
  P->prec = prec;
  const bool bf = (prec == KFAC_SKETCH_BF16);
  const bool sp = (prec == KFAC_SKETCH_SPLIT);
  size_t off = 0;
  auto take = [&](size_t bytes) { off = (off + kAlign - 1) / kAlign * kAlign; size_t o = off; off += bytes; return o; };
  // block steps of the grouped EA launches (one per activation precision) without split-K
  double ea_steps[2] = {0.0, 0.0};
  for (int i = 0; i < nf; ++i) {
    const kfac_factor_desc& F = factors[i];
    if (F.X == nullptr) continue;
    const int xb = (F.xtype == KFAC_BF16) ? 1 : 0;
    const double T = ea_tiles_per_side((int)F.d, xb == 1);
    ea_steps[xb] += T * (T + 1) / 2 * std::ceil((double)F.n / (xb ? 64.0 : 32.0));
  }
  for (int i = 0; i < nf; ++i) {
    const kfac_factor_desc& F = factors[i];
    FactorInfo I{};
    I.d = (int)F.d; I.r = (int)F.r; I.q = F.q;
    I.l = (int)std::min<int64_t>(F.r + F.p, F.d);
    I.l_pad = (int)round_up(I.l, 32);
    I.ldt = round_up(F.d, 8);
    I.exact = (I.l == I.d);
    I.ea = (F.X != nullptr);
    EigWs w(F.d, F.r, F.p, (int)prec, nullptr);
    I.ws_bytes = w.bytes;
    I.ws_off = take(w.bytes);
    const bool xb = (F.xtype == KFAC_BF16);
    I.ea_ks = I.ea ? ea_grouped_ksplit(I.d, F.n, xb, ea_steps[xb ? 1 : 0]) : 1;
    I.ea_bytes = I.ea ? ea_partial_bytes(I.d, I.ea_ks, xb) : 0;
    I.ea_off = take(I.ea_bytes + 16);
    I.sk_bytes = ((bf || sp) && !I.exact)
                     ? std::max(skinny_part_bytes(I.l_pad, I.d, I.d), split_part_bytes(I.l_pad, I.d, I.d)) : 0;
    I.sk_off = take(I.sk_bytes + 16);
    P->fi.push_back(I);
  }
  for (int l = 0; l < nl; ++l) {
    const kfac_layer_desc& L = layers[l];
    const int64_t dg = factors[L.fg].d, da = factors[L.fa].d, ra = factors[L.fa].r, rg = factors[L.fg].r;
    LayerInfo I{};
    const int ks1 = precondition_ksplit(dg, da, ra);
    I.bytes = kfac_precondition_workspace(dg, da, ra, rg) + (ks1 > 1 ? (size_t)ks1 * dg * ra * sizeof(float) + kAlign : 0);
    I.off = take(I.bytes);
    P->li.push_back(I);
  }
  // size the table head with every phase enabled, for either choice of the tunable kernels
  // and every branch count
  size_t tb = 0;
  for (int nb = 1; nb <= kMaxBranches; ++nb) {
    P->nbranch = nb;
    assign_branches(P, nb);
    for (int c = 0; c < 2; ++c) {
      Tables T;
      P->table_bytes = 0;
      P->gemm_cfg.assign(256, c);
      build_tables(P, nullptr, nullptr, T);
      tb = std::max(tb, T.bytes.size());
    }
  }
  P->nbranch = 1;
  assign_branches(P, 1);
  P->gemm_cfg.clear();
  P->table_bytes = (tb + 2 * kAlign) / kAlign * kAlign;
  P->ws_bytes = P->table_bytes + off + kAlign;
  *out = P;
  return KFAC_OK;
}

size_t kfac_plan_workspace(const kfac_plan* plan) { return plan ? plan->ws_bytes : 0; }

kfac_status kfac_plan_set_scalars(kfac_plan* plan, float rho, float lambda, uint64_t seed, uint32_t inversion_index,
                                  int do_ea, int do_eig, int do_precondition) {
  if (!plan || !(rho >= 0.f && rho < 1.f) || !(lambda > 0.f) || !std::isfinite(lambda)) return KFAC_EINVAL;
  plan->rho = rho; plan->lam = lambda; plan->seed = seed; plan->inv = inversion_index;
  plan->do_ea = do_ea != 0; plan->do_eig = do_eig != 0; plan->do_pre = do_precondition != 0;
  return KFAC_OK;
}

kfac_status kfac_plan_upload(kfac_plan* plan, void* workspace, size_t ws_bytes, int32_t* dev_status,
                             kfac_stream_t stream) {
  if (!plan || !workspace || !dev_status) return KFAC_EINVAL;
  if (ws_bytes < plan->ws_bytes) return KFAC_EWORKSPACE;
  Tables T;
  build_tables(plan, (char*)workspace, (int*)dev_status, T);
  if (T.bytes.size() > plan->table_bytes) return KFAC_EUNSUPPORTED;
  plan->tab = std::move(T);
  plan->dev = (char*)workspace;
  hipError_t e = hipMemcpyAsync(workspace, plan->tab.bytes.data(), plan->tab.bytes.size(), hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) return KFAC_EHIP;
  // the host copy must stay valid until the transfer has been consumed
  e = hipStreamSynchronize((hipStream_t)stream);
  return e == hipSuccess ? KFAC_OK : KFAC_EHIP;
}

int kfac_plan_launch_count(const kfac_plan* plan) { return plan ? (int)plan->tab.recs.size() : 0; }

const char* kfac_plan_launch_name(const kfac_plan* plan, int index) {
  static const char* names[] = {"ea_tiles", "ea_finalize", "ea_tiles_bf16", "ea_finalize_bf16", "omega",
                                "gemm_f32", "gemm_bf16", "gemm_bf16_skinny", "slice_reduce", "gemm_bf16x3", "gram_partial",
                                "gram_reduce", "cholinv", "trtri_cols", "trmm", "tridiag", "tri_prep", "tri_bisect",
                                "tri_select", "tri_vec", "tri_cluster_lead", "tri_cluster", "backtransform",
                                "sign_partial", "sign_apply", "gemm_f32_reduce"};
  static_assert(sizeof(names) / sizeof(names[0]) == K_GEMM_SL + 1, "one name per launch kind");
  if (!plan || index < 0 || index >= (int)plan->tab.recs.size()) return nullptr;
  return names[plan->tab.recs[index].kind];
}

kfac_status kfac_plan_launch_work(const kfac_plan* plan, int index, double* flops, double* bytes) {
  if (!plan || !flops || !bytes || index < 0 || index >= (int)plan->tab.recs.size()) return KFAC_EINVAL;
  *flops = plan->tab.recs[index].flops;
  *bytes = plan->tab.recs[index].bytes;
  return KFAC_OK;
}

namespace {
// Enqueues launch record r of the plan on stream s.
hipError_t launch_rec(const kfac_plan* plan, const LaunchRec& r, hipStream_t s) {
  char* d = plan->dev;
  {
    GroupMap gm{(const int*)(d + r.off_off), (const int*)(d + r.gx_off), r.ntasks};
    const void* tp = d + r.tasks_off;
    hipError_t e = hipSuccess;
    switch (r.kind) {
      case K_EA_TILES: e = launch_ea_tiles_g((const EaTask*)tp, gm, r.blocks, s); break;
      case K_EA_FIN: e = launch_ea_finalize_g((const EaTask*)tp, gm, r.blocks, s); break;
      case K_EA_TILES_BF: e = launch_ea_bf16_tiles_g((const EaTask*)tp, gm, r.blocks, s); break;
      case K_EA_FIN_BF: e = launch_ea_bf16_finalize_g((const EaTask*)tp, gm, r.blocks, s); break;
      case K_OMEGA: e = launch_omega_g((const OmegaTask*)tp, gm, r.blocks, s); break;
      case K_GEMM: e = launch_gemm_g((const GemmP*)tp, gm, r.blocks, r.ta, r.tb, r.cfg, r.split, s); break;
      case K_GEMM_SL: e = launch_gemm_slices_g((const GemmP*)tp, gm, r.blocks, s); break;
      case K_BF16: e = launch_gemm_bf16_g((const BfGemmTask*)tp, gm, r.blocks, s); break;
      case K_SKINNY: e = launch_skinny_g((const SkinnyTask*)tp, gm, r.blocks, s); break;
      case K_SKINNY_R: e = launch_reduce_g((const ReduceTask*)tp, gm, r.blocks, s); break;
      case K_SPLIT: e = launch_split_g((const SplitTask*)tp, gm, r.blocks, s); break;
      case K_GRAM_P: e = launch_gram_partial_g((const GramP*)tp, gm, r.blocks, s); break;
      case K_GRAM_R: e = launch_gram_reduce_g((const GramP*)tp, gm, r.blocks, s); break;
      case K_CHOLINV: e = launch_cholinv_g((const CholInvTask*)tp, gm, r.blocks, s); break;
      case K_TRTRI: e = launch_trtri_cols_g((const CholInvTask*)tp, gm, r.blocks, s); break;
      case K_TRMM: e = launch_trmm_g((const TrmmTask*)tp, gm, r.blocks, s); break;
      case K_TRIDIAG: e = launch_tridiag_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_PREP: e = launch_tri_prep_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_BISECT: e = launch_tri_bisect_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_SELECT: e = launch_tri_select_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_VEC: e = launch_tri_vec_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_CLEAD: e = launch_tri_cluster_lead_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_CLUSTER: e = launch_tri_cluster_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_BT: e = launch_backtransform_g((const EigTask*)tp, gm, r.blocks, s); break;
      case K_SIGN_P: e = launch_sign_partial_g((const SignTask*)tp, gm, r.blocks, s); break;
      case K_SIGN_A: e = launch_sign_apply_g((const SignTask*)tp, gm, r.blocks, s); break;
      default: return hipErrorInvalidValue;
    }
    return e;
  }
}
}  // namespace

kfac_status kfac_plan_launch_range(const kfac_plan* plan, int first, int count, kfac_stream_t stream) {
  if (!plan || !plan->dev || first < 0 || count < 0 || first + count > (int)plan->tab.recs.size())
    return KFAC_EINVAL;
  for (int i = first; i < first + count; ++i)
    if (launch_rec(plan, plan->tab.recs[i], (hipStream_t)stream) != hipSuccess) return KFAC_EHIP;
  return KFAC_OK;
}

kfac_status kfac_plan_launch(const kfac_plan* plan, kfac_stream_t stream) {
  if (!plan || !plan->dev) return KFAC_EINVAL;
  const int nb = plan->nbranch;
  if (nb <= 1) return kfac_plan_launch_range(plan, 0, (int)plan->tab.recs.size(), stream);
  // fork: branches 1.. wait for everything enqueued on the caller's stream so far
  hipStream_t s = (hipStream_t)stream;
  if (hipEventRecord(plan->fork, s) != hipSuccess) return KFAC_EHIP;
  for (int b = 1; b < nb; ++b)
    if (hipStreamWaitEvent(plan->stream[b - 1], plan->fork, 0) != hipSuccess) return KFAC_EHIP;
  // enqueue the branches' launches round-robin (each stream keeps its own order)
  std::vector<std::vector<const LaunchRec*>> per(nb + 1);
  for (const LaunchRec& r : plan->tab.recs) per[std::min(r.branch, nb)].push_back(&r);
  size_t longest = 0;
  for (int b = 0; b < nb; ++b) longest = std::max(longest, per[b].size());
  for (size_t k = 0; k < longest; ++k)
    for (int b = 0; b < nb; ++b)
      if (k < per[b].size() && launch_rec(plan, *per[b][k], b == 0 ? s : plan->stream[b - 1]) != hipSuccess)
        return KFAC_EHIP;
  // join, then the layers whose factors sit in different branches
  for (int b = 1; b < nb; ++b) {
    if (hipEventRecord(plan->join[b - 1], plan->stream[b - 1]) != hipSuccess) return KFAC_EHIP;
    if (hipStreamWaitEvent(s, plan->join[b - 1], 0) != hipSuccess) return KFAC_EHIP;
  }
  for (const LaunchRec* r : per[nb])
    if (launch_rec(plan, *r, s) != hipSuccess) return KFAC_EHIP;
  return KFAC_OK;
}

kfac_status kfac_plan_set_branches(kfac_plan* plan, int nbranch) {
  if (!plan || nbranch < 1 || nbranch > kMaxBranches) return KFAC_EINVAL;
  for (int b = 1; b < nbranch; ++b) {
    if (!plan->stream[b - 1] && hipStreamCreateWithFlags(&plan->stream[b - 1], hipStreamNonBlocking) != hipSuccess)
      return KFAC_EHIP;
    if (!plan->join[b - 1] && hipEventCreateWithFlags(&plan->join[b - 1], hipEventDisableTiming) != hipSuccess)
      return KFAC_EHIP;
  }
  if (nbranch > 1 && !plan->fork && hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming) != hipSuccess)
    return KFAC_EHIP;
  plan->nbranch = nbranch;
  assign_branches(plan, nbranch);
  plan->gemm_cfg.clear();       // the tunable launches are numbered anew
  return KFAC_OK;
}

int kfac_plan_launch_branch(const kfac_plan* plan, int index) {
  if (!plan || index < 0 || index >= (int)plan->tab.recs.size()) return -1;
  return plan->tab.recs[index].branch;
}

// ---- autotuner ---------------------------------------------------------------------------
namespace {

#ifndef KFAC_SRC_HASH
#define KFAC_SRC_HASH "unknown"
#endif

// What a stored timing is valid for: the library sources and build flags, the device
// architecture and the HIP runtime version.
uint64_t build_env_hash() {
  uint64_t h = 1469598103934665603ull;
  auto mixs = [&](const char* str) { for (; str && *str; ++str) { h ^= (unsigned char)*str; h *= 1099511628211ull; } };
  mixs(KFAC_SRC_HASH);
  int dev = 0, rt = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) mixs(prop.gcnArchName);
  if (hipRuntimeGetVersion(&rt) == hipSuccess) { h ^= (uint64_t)rt; h *= 1099511628211ull; }
  return h;
}

// Cache key of a tunable launch: the build / device / runtime hash, layout flags and every
// task's (M, N, K), hashed.
std::string gemm_key(const kfac_plan* P, const LaunchRec& r) {
  uint64_t h = build_env_hash();
  auto mix = [&](uint64_t v) { h ^= v; h *= 1099511628211ull; };
  mix((uint64_t)r.ta); mix((uint64_t)r.tb); mix((uint64_t)r.ntasks);
  const char* base = P->tab.bytes.data() + r.tasks_off;
  const bool f32 = (r.kind == K_GEMM);
  for (int i = 0; i < r.ntasks; ++i) {
    int M, N, K;
    if (f32) { const GemmP& t = ((const GemmP*)base)[i]; M = t.M; N = t.N; K = t.K; }
    else if (r.kind == K_BF16) { const BfGemmTask& t = ((const BfGemmTask*)base)[i]; M = t.M; N = t.N; K = t.K; }
    else { const SkinnyTask& t = ((const SkinnyTask*)base)[i]; M = t.M; N = t.N; K = t.K; }
    mix((uint64_t)M); mix((uint64_t)N); mix((uint64_t)K);
  }
  char buf[64];
  std::snprintf(buf, sizeof(buf), "%s:%016llx", f32 ? "gemm_f32" : "sketch_bf16", (unsigned long long)h);
  return buf;
}

std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> m;
  if (!path) return m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char key[128];
  int cfg;
  double us;
  while (std::fscanf(f, "%127s %d %lf", key, &cfg, &us) == 3)
    if (cfg >= 0 && cfg < 16) m[key] = cfg;
  std::fclose(f);
  return m;
}

}  // namespace

kfac_status kfac_plan_autotune(kfac_plan* plan, void* workspace, size_t ws_bytes, int32_t* dev_status,
                               const char* cache_path, int reps, kfac_stream_t stream) {
  if (!plan || !workspace || !dev_status || reps < 1) return KFAC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  kfac_status st = kfac_plan_upload(plan, workspace, ws_bytes, dev_status, stream);
  if (st != KFAC_OK) return st;
  int nord = 0;
  for (const LaunchRec& r : plan->tab.recs) nord = std::max(nord, r.ord + 1);
  plan->gemm_cfg.assign(nord, -1);
  std::map<std::string, int> cache = read_cache(cache_path);
  std::vector<std::string> lines;
  const char* ev = std::getenv("KFAC_AUTOTUNE_VERBOSE");
  const bool verbose = ev && ev[0] && ev[0] != '0';
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KFAC_EHIP;
  kfac_status result = KFAC_OK;
  for (int o = 0; o < nord && result == KFAC_OK; ++o) {
    // key of launch o with the configuration it currently has
    // key (independent of the configuration: the shapes) and number of configurations
    std::string key;
    int ncfg = 1;
    for (const LaunchRec& r : plan->tab.recs)
      if (r.ord == o) { key = gemm_key(plan, r); ncfg = r.ncfg; }
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second < ncfg) { plan->gemm_cfg[o] = hit->second; continue; }
    int best = 0;
    float best_ms = 1e30f;
    for (int c = 0; c < ncfg && result == KFAC_OK; ++c) {
      plan->gemm_cfg[o] = c;
      if ((result = kfac_plan_upload(plan, workspace, ws_bytes, dev_status, stream)) != KFAC_OK) break;
      int idx = -1, span = 1;
      for (size_t i = 0; i < plan->tab.recs.size(); ++i)
        if (plan->tab.recs[i].ord == o) { idx = (int)i; span = plan->tab.recs[i].span; }
      if (idx < 0) break;
      float tot = 0.f;
      for (int rep = 0; rep <= reps && result == KFAC_OK; ++rep) {   // rep 0 warms up
        if (hipEventRecord(e0, s) != hipSuccess) { result = KFAC_EHIP; break; }
        if ((result = kfac_plan_launch_range(plan, idx, span, stream)) != KFAC_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { result = KFAC_EHIP; break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tot += ms;
      }
      if (result == KFAC_OK && verbose) std::fprintf(stderr, "kfac autotune %s cfg %d: %.1f us\n", key.c_str(), c, 1e3 * tot / reps);
      if (result == KFAC_OK && tot / reps < best_ms) { best_ms = tot / reps; best = c; }
    }
    plan->gemm_cfg[o] = best;
    char line[192];
    std::snprintf(line, sizeof(line), "%s %d %.3f\n", key.c_str(), best, 1e3 * best_ms);
    lines.push_back(line);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (result != KFAC_OK) return result;
  if (cache_path && !lines.empty()) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      for (const std::string& l : lines) std::fputs(l.c_str(), f);
      std::fclose(f);
    }
  }
  return kfac_plan_upload(plan, workspace, ws_bytes, dev_status, stream);
}

kfac_status kfac_plan_force_config(kfac_plan* plan, int cfg_gemm_f32, int cfg_sketch_bf16) {
  if (!plan || cfg_gemm_f32 < -1 || cfg_gemm_f32 >= kGemmConfigs || cfg_sketch_bf16 < -1 || cfg_sketch_bf16 > 1)
    return KFAC_EINVAL;
  // walk the launch list once with defaults to learn which ordinal is which kind
  Tables T;
  plan->gemm_cfg.clear();
  build_tables(plan, nullptr, nullptr, T);
  int nord = 0;
  for (const LaunchRec& r : T.recs) nord = std::max(nord, r.ord + 1);
  plan->gemm_cfg.assign(nord, -1);
  for (const LaunchRec& r : T.recs) {
    if (r.ord < 0) continue;
    if (r.kind == K_GEMM && cfg_gemm_f32 >= 0 && cfg_gemm_f32 < r.ncfg) plan->gemm_cfg[r.ord] = cfg_gemm_f32;
    if ((r.kind == K_BF16 || r.kind == K_SKINNY) && cfg_sketch_bf16 >= 0) plan->gemm_cfg[r.ord] = cfg_sketch_bf16;
  }
  return KFAC_OK;
}

int kfac_plan_launch_config(const kfac_plan* plan, int index) {
  if (!plan || index < 0 || index >= (int)plan->tab.recs.size()) return -1;
  return plan->tab.recs[index].cfg;
}

void kfac_plan_destroy(kfac_plan* plan) {
  if (!plan) return;
  for (int b = 0; b < kMaxBranches - 1; ++b) {
    if (plan->stream[b]) (void)hipStreamDestroy(plan->stream[b]);
    if (plan->join[b]) (void)hipEventDestroy(plan->join[b]);
  }
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  delete plan;
}

}  // extern "C"
