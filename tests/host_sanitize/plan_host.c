/* Host-only exercise of the C ABI for the sanitizer build (AddressSanitizer +
 * UndefinedBehaviorSanitizer on the host code of libmsgfem): plans of
 * several shapes and decompositions (valid and rejected), both factor
 * layouts, every plan option, deflated rounds, coarse stores and their box
 * queries, errors, and destruction.  No call here touches a GPU: plan
 * creation, sizes, options and the coarse store's geometry are host-side (the
 * mesh arrays are only recorded, so placeholder pointers stand in for them).
 * Exit status 0 when every expectation holds; a sanitizer report aborts. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "msgfem.h"

static int failures = 0;
#define EXPECT(cond, what)                                 \
  do {                                                     \
    if (!(cond)) {                                         \
      fprintf(stderr, "FAILED: %s (line %d)\n", what, __LINE__); \
      ++failures;                                          \
    }                                                      \
  } while (0)

/* cores of a tensor decomposition of an nx x ny x nz mesh into cx x cy x cz
 * equal cores (the last ones take the remainder) */
static int tiles(int nx, int ny, int nz, int cx, int cy, int cz, int32_t *cores) {
  int n = 0;
  for (int k = 0; k < cz; ++k)
    for (int j = 0; j < cy; ++j)
      for (int i = 0; i < cx; ++i) {
        int32_t *c = cores + 6 * n++;
        c[0] = i * (nx / cx); c[3] = (i == cx - 1) ? nx : (i + 1) * (nx / cx);
        c[1] = j * (ny / cy); c[4] = (j == cy - 1) ? ny : (j + 1) * (ny / cy);
        c[2] = k * (nz / cz); c[5] = (k == cz - 1) ? nz : (k + 1) * (nz / cz);
      }
  return n;
}

static void check_plan(const char *name, msgfem_mesh *mesh, msgfem_decomp *dec, int nb, const int32_t *batch,
                       const int32_t *nev, const msgfem_eig_opts *opts) {
  msgfem_plan *p = NULL;
  int rc = msgfem_plan_create(&p, 0, mesh, dec, batch, nev, nb, opts);
  if (rc != MSGFEM_OK) {
    fprintf(stderr, "FAILED: %s: create %d: %s\n", name, rc, msgfem_plan_error(p));
    ++failures;
    msgfem_plan_destroy(p);
    return;
  }
  msgfem_sizes s, s2;
  EXPECT(msgfem_plan_sizes(p, &s) == MSGFEM_OK, "sizes");
  EXPECT(s.n_box == nb && s.block > 0 && s.ops_bytes > 0 && s.work_bytes > 0, "sizes content");
  for (int b = 0; b < nb; ++b) {
    msgfem_box_info bi;
    EXPECT(msgfem_plan_box(p, b, &bi) == MSGFEM_OK, "box");
    EXPECT(bi.n_dof == 3 * bi.n_nodes && bi.n1 > 0 && bi.n2 > 0 && bi.n1 + bi.n2 + bi.n3 <= bi.n_dof, "box dofs");
  }
  msgfem_box_info bad;
  EXPECT(msgfem_plan_box(p, nb, &bad) == MSGFEM_EARG, "box out of range");
  int64_t v = -1, nsplit = -1, fam = -1, bt = -1;
  EXPECT(msgfem_plan_get_option(p, MSGFEM_OPT_SPLIT, &v) == MSGFEM_OK && v == 1, "split default");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_INFO_SPLIT_BOXES, &nsplit) == MSGFEM_OK, "split boxes");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_INFO_SOLVE_FAMILY, &fam) == MSGFEM_OK && fam >= 5 && fam <= 15,
         "solve family");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_INFO_MAX_BT_AHAT, &bt) == MSGFEM_OK && bt >= 2, "max bt");
  /* the whole-band layout, back to the split one, every solve family */
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SPLIT, 0) == MSGFEM_OK, "split 0");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_INFO_SPLIT_BOXES, &v) == MSGFEM_OK && v == 0, "no split boxes");
  EXPECT(msgfem_plan_sizes(p, &s2) == MSGFEM_OK && s2.n_box == nb, "sizes after split 0");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SPLIT, 1) == MSGFEM_OK, "split 1");
  EXPECT(msgfem_plan_sizes(p, &s2) == MSGFEM_OK && s2.ops_bytes == s.ops_bytes && s2.work_bytes == s.work_bytes,
         "sizes restored");
  for (int f = 0; f <= 3; ++f) EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SOLVE, f) == MSGFEM_OK, "solve option");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SOLVE, 4) == MSGFEM_EARG, "solve option range");
  for (int f = 0; f <= 2; ++f) EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SPMM, f) == MSGFEM_OK, "spmm option");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_OPT_SPMM, &v) == MSGFEM_OK && v == 2, "spmm option read");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SPMM, 3) == MSGFEM_EARG, "spmm option range");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_SPMM, 0) == MSGFEM_OK, "spmm default");
  for (int f = 0; f <= 2; ++f) EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_CHOL, f) == MSGFEM_OK, "chol option");
  EXPECT(msgfem_plan_get_option(p, MSGFEM_OPT_CHOL, &v) == MSGFEM_OK && v == 2, "chol option read");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_CHOL, 3) == MSGFEM_EARG, "chol option range");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_CHOL, 0) == MSGFEM_OK, "chol default");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_GRAPH, 1) == MSGFEM_OK, "graph on");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_GRAPH, 2) == MSGFEM_EARG, "graph range");
  EXPECT(msgfem_plan_set_option(p, MSGFEM_OPT_GRAPH, 0) == MSGFEM_OK, "graph off");
  EXPECT(msgfem_plan_set_option(p, 77, 0) == MSGFEM_EARG, "unknown option");
  EXPECT(msgfem_plan_get_option(p, 77, &v) == MSGFEM_EARG, "unknown info");
  EXPECT(strlen(msgfem_plan_error(p)) > 0, "error text");
  printf("%s: %d boxes, block %d, ops %.3f GB, work %.3f GB, split boxes %lld, families %lld, widest Ahat band %lld\n",
         name, nb, s.block, s.ops_bytes / 1e9, s.work_bytes / 1e9, (long long)nsplit, (long long)fam,
         (long long)bt);
  msgfem_plan_destroy(p);
}

int main(void) {
  /* placeholder mesh arrays: recorded by the plan, never read on the host */
  void *fake = (void *)(uintptr_t)0x1000;
  static int32_t cores[6 * 512], ovs[512], nev[512], batch[512];
  /* a beam-like mesh and a laminate-like mesh with cubic cores */
  struct { const char *name; int nx, ny, nz, cx, cy, cz, overlap, ovs, nev, nmat; } cases[] = {
      {"beam 48x6x6, 4 cores", 48, 6, 6, 4, 1, 1, 2, 2, 10, 2},
      {"laminate 96x64x48, 16^3 cores", 96, 64, 48, 6, 4, 3, 2, 2, 20, 4},
      {"cube 24^3, 27 cores", 24, 24, 24, 3, 3, 3, 1, 1, 44, 3},
  };
  for (unsigned c = 0; c < sizeof cases / sizeof cases[0]; ++c) {
    msgfem_mesh mesh = {cases[c].nx, cases[c].ny, cases[c].nz, cases[c].nmat, fake, fake, fake, fake};
    int nsd = tiles(cases[c].nx, cases[c].ny, cases[c].nz, cases[c].cx, cases[c].cy, cases[c].cz, cores);
    for (int j = 0; j < nsd; ++j) {
      ovs[j] = cases[c].ovs;
      nev[j] = cases[c].nev;
      batch[j] = j;
    }
    msgfem_decomp dec = {nsd, cores, cases[c].overlap, ovs};
    msgfem_eig_opts opts = {1.0, 1e-6, 200, 0, 0, 0, 1234};
    check_plan(cases[c].name, &mesh, &dec, nsd, batch, nev, &opts);
    opts.precision = 1;
    check_plan(cases[c].name, &mesh, &dec, nsd, batch, nev, &opts);
    opts.precision = 0;
    opts.geneo = 1;
    if (cases[c].nev <= 32) check_plan(cases[c].name, &mesh, &dec, nsd, batch, nev, &opts);
    /* coarse stores over the whole decomposition */
    for (int geneo = 0; geneo < 2; ++geneo) {
      msgfem_coarse *cs = NULL;
      int rc = msgfem_coarse_create(&cs, 0, &mesh, &dec, nev, geneo);
      EXPECT(rc == MSGFEM_OK, "coarse create");
      if (rc == MSGFEM_OK) {
        int64_t bytes = 0, off = 0;
        int32_t nh = 0, ncol = 0, ndof = 0, roff = 0;
        EXPECT(msgfem_coarse_store_sizes(cs, &bytes, &nh, &ncol) == MSGFEM_OK && bytes > 0 && nh > 0, "store sizes");
        for (int j = 0; j < nsd; ++j)
          EXPECT(msgfem_coarse_box(cs, j, &off, &ndof, &roff) == MSGFEM_OK && ndof > 0, "store box");
        EXPECT(msgfem_coarse_box(cs, nsd, &off, &ndof, &roff) == MSGFEM_EARG, "store box range");
      } else {
        fprintf(stderr, "  %s\n", msgfem_coarse_error(cs));
      }
      msgfem_coarse_destroy(cs);
    }
    /* rejected plans: no boxes, n_ev beyond 48, block 24 with n_ev > 32, a core outside the mesh */
    msgfem_plan *p = NULL;
    EXPECT(msgfem_plan_create(&p, 0, &mesh, &dec, batch, nev, 0, &opts) == MSGFEM_EARG, "nb 0");
    msgfem_plan_destroy(p);
    p = NULL;
    int32_t big[1] = {49};
    EXPECT(msgfem_plan_create(&p, 0, &mesh, &dec, batch, big, 1, NULL) == MSGFEM_EARG, "n_ev 49");
    msgfem_plan_destroy(p);
    p = NULL;
    int32_t forty[1] = {40};
    msgfem_eig_opts o24 = {1.0, 1e-6, 200, 24, 0, 0, 1};
    EXPECT(msgfem_plan_create(&p, 0, &mesh, &dec, batch, forty, 1, &o24) == MSGFEM_EARG, "block 24 with rounds");
    msgfem_plan_destroy(p);
    p = NULL;
    int32_t save = cores[3];
    cores[3] = cases[c].nx + 5;
    EXPECT(msgfem_plan_create(&p, 0, &mesh, &dec, batch, nev, 1, NULL) == MSGFEM_EARG, "core out of mesh");
    cores[3] = save;
    msgfem_plan_destroy(p);
  }
  EXPECT(msgfem_static_scratch_max() == 16 << 20, "static scratch size");
  if (failures) fprintf(stderr, "%d failures\n", failures);
  else printf("all host checks passed\n");
  return failures ? 1 : 0;
}
