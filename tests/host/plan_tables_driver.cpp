// Driver of the host-only sanitizer build of the plan-table code (tests/test_host_sanitizers.py):
// reads plan cases from a text file, runs rpa_plan_create (tables in host memory), checks the
// status against the expected one, prints a summary of the tables, sets tau points per launch to
// all of them, prints the summary again and destroys the plan.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/rpa_mi355x.h"

extern "C" rpa_ctx *rpa_test_host_ctx(void);
extern "C" void rpa_test_host_ctx_free(rpa_ctx *ctx);
extern "C" int rpa_test_plan_summary(const rpa_plan *p, long long *out);

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  FILE *f = std::fopen(argv[1], "r");
  if (!f) return 2;
  rpa_ctx *ctx = rpa_test_host_ctx();
  char name[128];
  int expect, natoms, ntau, prec, mesh[3];
  int ncases = 0;
  while (std::fscanf(f, " case %127s %d %d %d %d %d %d %d", name, &expect, &natoms, &ntau, &prec, &mesh[0], &mesh[1],
                     &mesh[2]) == 8) {
    std::vector<int> nao(natoms), naux(natoms);
    for (int &x : nao)
      if (std::fscanf(f, "%d", &x) != 1) return 3;
    for (int &x : naux)
      if (std::fscanf(f, "%d", &x) != 1) return 3;
    int nblk = 0;
    if (std::fscanf(f, "%d", &nblk) != 1) return 3;
    std::vector<int> I(nblk), K(nblk), R(3 * nblk);
    std::vector<long long> off(nblk);
    for (int b = 0; b < nblk; ++b)
      if (std::fscanf(f, "%d %d %d %d %d %lld", &I[b], &K[b], &R[3 * b], &R[3 * b + 1], &R[3 * b + 2], &off[b]) != 6)
        return 3;
    rpa_cell cell{natoms, nao.data(), naux.data(), {mesh[0], mesh[1], mesh[2]}};
    rpa_lri_blocks blocks{nblk, I.data(), K.data(), R.data(), off.data()};
    rpa_plan *plan = nullptr;
    size_t ws = 0;
    const int rc = rpa_plan_create(ctx, &cell, &blocks, ntau, prec, &ws, &plan);
    if (rc != expect) {
      std::printf("case %s: status %d, expected %d (%s)\n", name, rc, expect, rpa_last_error(ctx));
      return 1;
    }
    if (rc == RPA_OK) {
      long long s[8];
      rpa_test_plan_summary(plan, s);
      std::printf("summary %s %lld %lld %lld %lld %lld %lld %lld %lld\n", name, s[0], s[1], s[2], s[3], s[4], s[5],
                  s[6], s[7]);
      size_t ws2 = 0;
      if (rpa_plan_set_tau_batch(plan, ntau, &ws2) != RPA_OK || ws2 < ws) return 4;
      rpa_test_plan_summary(plan, s);
      std::printf("batched %s %lld\n", name, s[0]);
      rpa_plan_destroy(plan);
    }
    ++ncases;
  }
  std::fclose(f);
  rpa_test_host_ctx_free(ctx);
  std::printf("cases %d\n", ncases);
  return 0;
}
