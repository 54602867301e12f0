// Drives every entry point of the CPU oracle on small random inputs, for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure: tests/test_sanitize.py compiles and runs it).  Exits 0
// when every call succeeds and the self-checks hold; the sanitizers abort
// on the first invalid access or undefined operation.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_spgemm(int sr, int vt, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                  const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t ncols, const int64_t* cols,
                  int64_t* counts, const int64_t* offs, int32_t* cir, void* cnum, int nthreads);
int64_t oracle_spgemm_check(int sr, int vt, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                            const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t j0, int64_t j1,
                            const int64_t* gcp, const int32_t* gir, const void* gnum, double rtol,
                            int64_t* first_bad, int nthreads);
int oracle_spref(int64_t m, const int64_t* acp, const int32_t* air, const void* anum, int vbytes, int64_t lenI,
                 const int32_t* I, int64_t lenJ, const int32_t* J, int64_t* counts, const int64_t* offs,
                 int32_t* bir, void* bnum, int nthreads);
int oracle_spasgn(int64_t m, int64_t n, const int64_t* acp, const int32_t* air, const void* anum, int vbytes,
                  int64_t lenI, const int32_t* I, int64_t lenJ, const int32_t* J, const int64_t* bcp,
                  const int32_t* bir, const void* bnum, int64_t* counts, const int64_t* offs, int32_t* cir,
                  void* cnum, int nthreads);
int oracle_extend_add(int sr, int vt, int64_t m, int64_t n, const int64_t* acp, const int32_t* air,
                      const void* anum, int64_t lenI, const int32_t* I, int64_t lenJ, const int32_t* J,
                      const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t* counts,
                      const int64_t* offs, int32_t* cir, void* cnum, int nthreads);
int64_t oracle_csc_to_dcsc(int64_t n, const int64_t* cp, int32_t* jc, int64_t* dcp);
}

namespace {

struct Csc {
  int64_t m = 0, n = 0;
  std::vector<int64_t> cp;
  std::vector<int32_t> ir;
  std::vector<double> num;
  std::vector<int64_t> inum;
};

Csc random_csc(std::mt19937_64& rng, int64_t m, int64_t n, double density) {
  Csc a;
  a.m = m;
  a.n = n;
  a.cp.assign(n + 1, 0);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = 0; i < m; ++i)
      if (u(rng) * 0.5 + 0.5 < density) {
        a.ir.push_back((int32_t)i);
        a.num.push_back(u(rng));
        a.inum.push_back((int64_t)(rng() % 7) - 3);
      }
    a.cp[j + 1] = (int64_t)a.ir.size();
  }
  return a;
}

std::vector<int64_t> offsets(const std::vector<int64_t>& counts) {
  std::vector<int64_t> off(counts.size() + 1, 0);
  for (size_t t = 0; t < counts.size(); ++t) off[t + 1] = off[t] + counts[t];
  return off;
}

int fails = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s\n", what);
    ++fails;
  }
}

void product(const Csc& A, const Csc& B, int sr, bool ints, int threads) {
  const int vt = ints ? 2 : 1;
  const void* an = ints ? (const void*)A.inum.data() : (const void*)A.num.data();
  const void* bn = ints ? (const void*)B.inum.data() : (const void*)B.num.data();
  std::vector<int64_t> counts(B.n);
  expect(oracle_spgemm(sr, vt, A.m, A.cp.data(), A.ir.data(), an, B.cp.data(), B.ir.data(), bn, B.n, nullptr,
                       counts.data(), nullptr, nullptr, nullptr, threads) == 0, "spgemm count");
  const std::vector<int64_t> off = offsets(counts);
  std::vector<int32_t> cir(off.back() + 1);
  std::vector<double> cd(off.back() + 1);
  std::vector<int64_t> ci(off.back() + 1);
  void* cn = ints ? (void*)ci.data() : (void*)cd.data();
  expect(oracle_spgemm(sr, vt, A.m, A.cp.data(), A.ir.data(), an, B.cp.data(), B.ir.data(), bn, B.n, nullptr,
                       nullptr, off.data(), cir.data(), cn, threads) == 0, "spgemm fill");
  int64_t first = 0;
  expect(oracle_spgemm_check(sr, vt, A.m, A.cp.data(), A.ir.data(), an, B.cp.data(), B.ir.data(), bn, 0, B.n,
                             off.data(), cir.data(), cn, 1e-12, &first, threads) == 0, "spgemm self-check");
  // a subset of columns, in an order of its own
  std::vector<int64_t> cols;
  for (int64_t j = B.n - 1; j >= 0; j -= 3) cols.push_back(j);
  std::vector<int64_t> sc(cols.size());
  expect(oracle_spgemm(sr, vt, A.m, A.cp.data(), A.ir.data(), an, B.cp.data(), B.ir.data(), bn,
                       (int64_t)cols.size(), cols.data(), sc.data(), nullptr, nullptr, nullptr, threads) == 0,
         "spgemm column subset");
  // pattern only
  expect(oracle_spgemm(3, 3, A.m, A.cp.data(), A.ir.data(), nullptr, B.cp.data(), B.ir.data(), nullptr, B.n,
                       nullptr, counts.data(), nullptr, nullptr, nullptr, threads) == 0, "spgemm pattern");
}

}  // namespace

int main() {
  std::mt19937_64 rng(12345);
  for (int trial = 0; trial < 6; ++trial) {
    const int64_t m = 1 + (int64_t)(rng() % 60), k = 1 + (int64_t)(rng() % 60), n = (int64_t)(rng() % 60);
    const Csc A = random_csc(rng, m, k, 0.15);
    const Csc B = random_csc(rng, k, n, 0.15);
    const int threads = 1 + trial % 3;
    for (int sr : {0, 1, 2, 4}) {
      product(A, B, sr, false, threads);
      product(A, B, sr, true, threads);
    }
    // SpRef with repeats
    std::vector<int32_t> I, J;
    for (int t = 0; t < 40; ++t) I.push_back((int32_t)(rng() % m));
    for (int t = 0; t < 30; ++t) J.push_back((int32_t)(rng() % k));
    std::vector<int64_t> rc(J.size());
    expect(oracle_spref(m, A.cp.data(), A.ir.data(), A.num.data(), 8, (int64_t)I.size(), I.data(),
                        (int64_t)J.size(), J.data(), rc.data(), nullptr, nullptr, nullptr, threads) == 0, "spref");
    std::vector<int64_t> ro = offsets(rc);
    std::vector<int32_t> rir(ro.back() + 1);
    std::vector<double> rnum(ro.back() + 1);
    expect(oracle_spref(m, A.cp.data(), A.ir.data(), A.num.data(), 8, (int64_t)I.size(), I.data(),
                        (int64_t)J.size(), J.data(), nullptr, ro.data(), rir.data(), rnum.data(), threads) == 0,
           "spref fill");
    // SpAsgn and extend-add of a block of the index sizes
    const Csc Bs = random_csc(rng, (int64_t)I.size(), (int64_t)J.size(), 0.2);
    std::vector<int64_t> ac(k);
    expect(oracle_spasgn(m, k, A.cp.data(), A.ir.data(), A.num.data(), 8, (int64_t)I.size(), I.data(),
                         (int64_t)J.size(), J.data(), Bs.cp.data(), Bs.ir.data(), Bs.num.data(), ac.data(), nullptr,
                         nullptr, nullptr, threads) == 0, "spasgn");
    std::vector<int64_t> ao = offsets(ac);
    std::vector<int32_t> air2(ao.back() + 1);
    std::vector<double> anum2(ao.back() + 1);
    expect(oracle_spasgn(m, k, A.cp.data(), A.ir.data(), A.num.data(), 8, (int64_t)I.size(), I.data(),
                         (int64_t)J.size(), J.data(), Bs.cp.data(), Bs.ir.data(), Bs.num.data(), nullptr, ao.data(),
                         air2.data(), anum2.data(), threads) == 0, "spasgn fill");
    for (int sr : {0, 1, 3}) {
      const int vt = sr == 3 ? 3 : 1;
      std::vector<int64_t> ec(k);
      expect(oracle_extend_add(sr, vt, m, k, A.cp.data(), A.ir.data(), A.num.data(), (int64_t)I.size(), I.data(),
                               (int64_t)J.size(), J.data(), Bs.cp.data(), Bs.ir.data(), Bs.num.data(), ec.data(),
                               nullptr, nullptr, nullptr, threads) == 0, "extend-add");
      std::vector<int64_t> eo = offsets(ec);
      std::vector<int32_t> eir(eo.back() + 1);
      std::vector<double> enm(eo.back() + 1);
      expect(oracle_extend_add(sr, vt, m, k, A.cp.data(), A.ir.data(), A.num.data(), (int64_t)I.size(), I.data(),
                               (int64_t)J.size(), J.data(), Bs.cp.data(), Bs.ir.data(), Bs.num.data(), nullptr,
                               eo.data(), eir.data(), vt == 3 ? nullptr : enm.data(), threads) == 0,
             "extend-add fill");
    }
    // an index out of range is refused, not read
    std::vector<int32_t> bad = I;
    bad.push_back((int32_t)m);
    expect(oracle_spref(m, A.cp.data(), A.ir.data(), A.num.data(), 8, (int64_t)bad.size(), bad.data(),
                        (int64_t)J.size(), J.data(), rc.data(), nullptr, nullptr, nullptr, threads) != 0,
           "spref rejects a bad index");
    const int64_t nzc = oracle_csc_to_dcsc(k, A.cp.data(), nullptr, nullptr);
    std::vector<int32_t> jc(nzc + 1);
    std::vector<int64_t> dcp(nzc + 1);
    expect(oracle_csc_to_dcsc(k, A.cp.data(), jc.data(), dcp.data()) == nzc, "csc to dcsc");
  }
  if (fails) return 1;
  std::printf("oracle under sanitizers: ok\n");
  return 0;
}
