// Pairwise tensor contraction planner: out(lo) = A(la) * B(lb).
//
// Labels are single characters.  Contracted labels (in la and lb, not in lo)
// form the GEMM's K; the free labels of A and of B keep their order and form
// M and N.  An operand whose legs are already [free, K] or [K, free] feeds the
// GEMM directly (as op or op^T); otherwise it is permuted first.  The GEMM
// result is [free_A, free_B]; it is permuted once more only if lo differs.
#include <cstring>
#include <stdexcept>
#include <string>

#include "ctm_internal.h"

namespace ctm {

static int64_t dim_of(const Tensor& t, const std::string& labs, char l) {
  const size_t i = labs.find(l);
  if (i == std::string::npos) throw std::runtime_error("label not found");
  return t.dims[i];
}

Tensor relabel(Ctx& c, const Tensor& A, const char* la, const char* lo, int out_dt) {
  const std::string sa(la), so(lo);
  if ((int)sa.size() != A.nd || so.size() != sa.size())
    throw std::runtime_error("relabel: rank mismatch " + sa + " -> " + so);
  if (sa == so && A.dt == out_dt) return A;
  int perm[kMaxDims];
  std::vector<int64_t> dims;
  for (size_t i = 0; i < so.size(); ++i) {
    const size_t j = sa.find(so[i]);
    if (j == std::string::npos) throw std::runtime_error("relabel: missing label");
    perm[i] = (int)j;
    dims.push_back(A.dims[j]);
  }
  Tensor out = c.alloc(out_dt, dims);
  permute(c, A, perm, out);
  return out;
}

Tensor contract(Ctx& c, const Tensor& A, const char* la, const Tensor& B, const char* lb,
                const char* lo, int compute, int out_dt) {
  const std::string sa(la), sb(lb), so(lo);
  if ((int)sa.size() != A.nd || (int)sb.size() != B.nd)
    throw std::runtime_error("contract: rank mismatch " + sa + "," + sb);
  std::string K, fa, fb;
  for (char l : sa) {
    const bool inb = sb.find(l) != std::string::npos, ino = so.find(l) != std::string::npos;
    if (inb && ino) throw std::runtime_error("contract: batch label unsupported");
    if (!inb && !ino) throw std::runtime_error("contract: trace label unsupported");
    if (inb) K += l; else fa += l;
  }
  for (char l : sb) {
    const bool ina = sa.find(l) != std::string::npos, ino = so.find(l) != std::string::npos;
    if (!ina && !ino) throw std::runtime_error("contract: trace label unsupported");
    if (!ina) fb += l;
  }
  for (size_t i = 0; i < K.size(); ++i)
    if (dim_of(A, sa, K[i]) != dim_of(B, sb, K[i])) throw std::runtime_error("contract: dim mismatch");
  int64_t M = 1, N = 1, KK = 1;
  for (char l : fa) M *= dim_of(A, sa, l);
  for (char l : fb) N *= dim_of(B, sb, l);
  for (char l : K) KK *= dim_of(A, sa, l);

  auto a_ok = [&](const std::string& k, int* ta) {
    if (A.dt != compute) return false;
    if (sa == fa + k) { *ta = 0; return true; }
    if (sa == k + fa) { *ta = 1; return true; }
    return false;
  };
  auto b_ok = [&](const std::string& k, int* tb) {
    if (B.dt != compute) return false;
    if (sb == k + fb) { *tb = 0; return true; }
    if (sb == fb + k) { *tb = 1; return true; }
    return false;
  };
  // K order: A's, unless A needs a permute anyway and B already fits its own
  std::string Kb;
  for (char l : sb)
    if (K.find(l) != std::string::npos) Kb += l;
  int ta = 0, tb = 0;
  Tensor Aop = A, Bop = B;
  std::string Ko = K;
  if (a_ok(K, &ta)) {
    if (!b_ok(K, &tb)) { Bop = relabel(c, B, lb, (K + fb).c_str(), compute); tb = 0; }
  } else if (b_ok(Kb, &tb)) {
    Ko = Kb;
    Aop = relabel(c, A, la, (fa + Kb).c_str(), compute);
    ta = 0;
  } else {
    Aop = relabel(c, A, la, (fa + K).c_str(), compute);
    ta = 0;
    Bop = relabel(c, B, lb, (K + fb).c_str(), compute);
    tb = 0;
  }
  const int64_t lda = ta ? M : KK;
  const int64_t ldb = tb ? KK : N;
  const int gdt = compute == F64 ? F64 : F32;
  const std::string cl = fa + fb;
  std::vector<int64_t> cdims;
  for (char l : fa) cdims.push_back(dim_of(A, sa, l));
  for (char l : fb) cdims.push_back(dim_of(B, sb, l));
  if (so.size() != cl.size()) throw std::runtime_error("contract: output labels");
  if (M > 0x7fffffff || N > 0x7fffffff || KK > 0x7fffffff)
    throw std::runtime_error("contract: GEMM dimension too large");
  if (cl == so && gdt == out_dt) {
    Tensor out = c.alloc(out_dt, cdims);
    gemm(c, compute, (int)M, (int)N, (int)KK, 1.0, Aop.p, lda, ta, Bop.p, ldb, tb, 0.0, out.p, N);
    return out;
  }
  Tensor tmp = c.alloc(gdt, cdims);
  gemm(c, compute, (int)M, (int)N, (int)KK, 1.0, Aop.p, lda, ta, Bop.p, ldb, tb, 0.0, tmp.p, N);
  return relabel(c, tmp, cl.c_str(), lo, out_dt);
}

}  // namespace ctm
