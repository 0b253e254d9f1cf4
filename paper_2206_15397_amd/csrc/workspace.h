// Workspace layouts shared by the single-factor entry points and the grouped plan.
#pragma once
#include <algorithm>
#include "kernels.h"

namespace kfac {

constexpr size_t kAlign = 256;

struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }


// Layout of the kfac_rand_eig workspace; with base == nullptr it only measures.
struct EigWs {
  int64_t d, r, l, l_pad, ldt;
  bool exact, bf16, split;
  float *OmT, *Yt, *Qt, *P, *sval;
  int* sidx;
  uint16_t *OmTb, *Qtb;
  double *G, *Wc, *Li, *part, *A, *V, *diag, *off, *Z, *scr, *Dd;
  float* skp;            // bf16 mode, l_pad <= 288: split-K partials of the whole-width GEMMs
  int* fail;
  size_t bytes;

  // prec: KFAC_SKETCH_FP32 / _BF16 (bf16 copies of Omega^T and Q^T) / _SPLIT (fp32 only)
  EigWs(int64_t d_, int64_t r_, int64_t p_, int prec, void* base)
      : d(d_), r(r_), bf16(prec == KFAC_SKETCH_BF16), split(prec == KFAC_SKETCH_SPLIT) {
    l = std::min<int64_t>(r + p_, d);
    exact = (l == d);
    l_pad = round_up(l, 32);
    ldt = round_up(d, 8);
    Bump b(base);
    const int64_t n = exact ? d : l;
    OmT = Yt = Qt = P = nullptr;
    OmTb = Qtb = nullptr;
    G = Wc = Li = part = nullptr;
    skp = nullptr;
    if (!exact) {
      OmT = b.take<float>(l_pad * ldt);
      Yt = b.take<float>(l_pad * ldt);
      Qt = b.take<float>(l_pad * ldt);
      if (bf16) {
        OmTb = b.take<uint16_t>(l_pad * ldt);
        Qtb = b.take<uint16_t>(l_pad * ldt);
      }
      if (bf16 || split) {
        if (l_pad <= kWholeWidthMaxM) {
          const size_t pb = std::max(skinny_part_bytes((int)l_pad, (int)d, (int)d),
                                     split_part_bytes((int)l_pad, (int)d, (int)d));
          skp = b.take<float>(pb / sizeof(float) + 4);
        }
      }
      G = b.take<double>(l_pad * l_pad);
      Wc = b.take<double>(l_pad * l_pad);
      Li = b.take<double>(l_pad * 16);
      size_t pb = std::max(gram_workspace_bytes((int)l_pad, (int)d, 1), gram_workspace_bytes((int)l_pad, (int)d, 0));
      part = b.take<double>(pb / sizeof(double) + 1);
      P = b.take<float>(l_pad * r);
    }
    A = b.take<double>(n * n);
    V = b.take<double>(n * n);
    diag = b.take<double>(n + 1);
    off = b.take<double>(n + 1);
    Z = b.take<double>(n * r);
    scr = b.take<double>(small_eig_scratch_doubles((int)n, (int)r));
    Dd = b.take<double>(r);
    sval = b.take<float>((size_t)sign_chunks((int)d) * r);
    sidx = b.take<int>((size_t)sign_chunks((int)d) * r);
    fail = b.take<int>(16);
    bytes = b.off + kAlign;
  }
};


}  // namespace kfac
