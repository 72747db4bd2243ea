/* Host-side checks of libtgp's entry points, built with AddressSanitizer.
 *
 * Every call here fails a host-side argument check before any device work
 * (pointers are never dereferenced), or exercises host-only code (status
 * strings, the autotune cache file parser and writer), so the program runs
 * without a GPU. It returns 0 when every call gave the expected status; the
 * sanitizer reports any out-of-bounds access or leak in the host code. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tgp.h"

static int g_fail = 0;

#define EXPECT(call, want)                                                                    \
  do {                                                                                        \
    const int got_ = (int)(call);                                                             \
    if (got_ != (int)(want)) {                                                                \
      fprintf(stderr, "%s:%d: %s gave %d, expected %d\n", __FILE__, __LINE__, #call, got_,    \
              (int)(want));                                                                   \
      g_fail = 1;                                                                             \
    }                                                                                         \
  } while (0)

#define FAKE(k) ((void*)(uintptr_t)(0x10000u * (k)))

static tgp_pop pop(int64_t P, int32_t Lmax, int64_t stride) {
  tgp_pop p = {(const float*)FAKE(1), (const float*)FAKE(2), (const float*)FAKE(3), P, Lmax, stride};
  return p;
}

static tgp_data data(int32_t V, int64_t D, int32_t n_out, const void* Y) {
  tgp_data d = {(const float*)FAKE(4), V, D, D, (const float*)Y, n_out, D};
  return d;
}

static void write_file(const char* path, const char* text) {
  FILE* f = fopen(path, "w");
  if (!f) {
    perror(path);
    exit(2);
  }
  fputs(text, f);
  fclose(f);
}

static void evaluation_calls(void) {
  tgp_pop p = pop(10, 64, 64);
  tgp_data d = data(2, 100, 1, FAKE(5));
  float* mse = (float*)FAKE(6);
  EXPECT(tgp_workspace_bytes(NULL, &d, 1, 0) == 0, 1);
  EXPECT(tgp_workspace_bytes(&p, &d, 1, 0) > 0, 1);
  EXPECT(tgp_workspace_bytes(&p, &d, 1, 1) > 0, 1);
  tgp_pop big = pop(10, 2048, 2048);
  EXPECT(tgp_workspace_bytes(&big, &d, 1, 0) == 0, 1);
  EXPECT(tgp_eval_mse(NULL, &d, NULL, mse, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  EXPECT(tgp_eval_mse(&p, NULL, NULL, mse, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  EXPECT(tgp_eval_mse(&p, &d, NULL, NULL, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  EXPECT(tgp_eval_mse(&big, &d, NULL, mse, NULL, FAKE(7), 1 << 20, NULL), TGP_E_UNSUPPORTED);
  tgp_pop narrow = pop(10, 64, 10);
  EXPECT(tgp_eval_mse(&narrow, &d, NULL, mse, NULL, FAKE(7), 1 << 20, NULL), TGP_E_SHAPE);
  tgp_data wide = data(17, 100, 1, FAKE(5));
  EXPECT(tgp_eval_mse(&p, &wide, NULL, mse, NULL, FAKE(7), 1 << 20, NULL), TGP_E_UNSUPPORTED);
  EXPECT(tgp_eval_mse(&p, &d, NULL, mse, NULL, NULL, 0, NULL), TGP_E_WORKSPACE);
  EXPECT(tgp_eval_mse(&p, &d, NULL, mse, NULL, FAKE(7), 64, NULL), TGP_E_WORKSPACE);
  EXPECT(tgp_eval_mse_noalloc(NULL, &d, NULL, mse, NULL, NULL), TGP_E_ARG);
  EXPECT(tgp_eval_mse_noalloc(&narrow, &d, NULL, mse, NULL, NULL), TGP_E_SHAPE);
  tgp_pop huge = pop(200000, 1024, 1024);
  tgp_data d4 = data(4, 4096, 1, FAKE(5));
  EXPECT(tgp_eval_mse_noalloc(&huge, &d4, NULL, mse, NULL, NULL), TGP_E_TOO_LARGE);
  tgp_data many = data(2, 100, 13, FAKE(5));
  EXPECT(tgp_eval_multi_output(&p, &many, NULL, mse, NULL, 0, NULL, FAKE(7), 1 << 20, NULL), TGP_E_UNSUPPORTED);
  tgp_data three = data(2, 100, 3, FAKE(5));
  EXPECT(tgp_eval_multi_output(&p, &three, NULL, NULL, NULL, 0, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  EXPECT(tgp_eval_accuracy(&p, &three, NULL, NULL, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  tgp_data five = data(2, 100, 5, FAKE(5));
  EXPECT(tgp_eval_mse_grad(&p, &five, NULL, NULL, mse, NULL, NULL, NULL, FAKE(7), 1 << 20, NULL),
         TGP_E_UNSUPPORTED);
  EXPECT(tgp_plan(NULL, 2, 1, NULL, NULL, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  tgp_cfg out;
  int32_t found = -1;
  EXPECT(tgp_autotune(&p, &d, 1, 0, NULL, FAKE(7), 1 << 20, NULL), TGP_E_ARG);
  EXPECT(tgp_autotune(&p, &d, 1, 1, &out, FAKE(7), 64, NULL), TGP_E_WORKSPACE);
  EXPECT(tgp_autotune_cached(&p, &d, 1, 0, NULL, &found), TGP_E_ARG);
  EXPECT(tgp_autotune_cached(&p, &d, 1, 0, &out, NULL), TGP_E_ARG);
  EXPECT(tgp_autotune_cached(&big, &d, 1, 0, &out, &found), TGP_E_UNSUPPORTED);
  EXPECT(tgp_autotune_cached(&p, &d, 5, 1, &out, &found), TGP_E_UNSUPPORTED);
}

static void exchange_and_generation_calls(void) {
  tgp_pop p = pop(10, 64, 64);
  tgp_exchange x = {NULL, FAKE(8), NULL, NULL, 5, 64, 0};
  float* o = (float*)FAKE(64);
  EXPECT(tgp_subtree_exchange(&p, &p, NULL, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_ARG);
  x.flags = 8;
  EXPECT(tgp_subtree_exchange(&p, &p, &x, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_ARG);
  x.flags = 0;
  x.max_len = 65;
  EXPECT(tgp_subtree_exchange(&p, &p, &x, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_SHAPE);
  x.max_len = 64;
  EXPECT(tgp_subtree_exchange(&p, &p, &x, o, o + 4096, o + 8192, 63, NULL, NULL), TGP_E_SHAPE);
  x.B = 0;
  x.old_node = NULL;
  EXPECT(tgp_subtree_exchange(&p, &p, &x, NULL, NULL, NULL, 64, NULL, NULL), TGP_OK);
  const int32_t funcs[3] = {0, 1, 2};
  const int32_t dup[2] = {1, 1};
  tgp_gen_cfg g = {TGP_GEN_RAMPED, 2, 6, 2, funcs, 3, -5.0f, 5.0f, -1.0f, -1.0f, 8, 1u, 0};
  EXPECT(tgp_generate(NULL, 1, 8, o, o, o, 8, NULL, NULL), TGP_E_ARG);
  EXPECT(tgp_generate(&g, -1, 64, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_SHAPE);
  g.depth_max = 31;
  EXPECT(tgp_generate(&g, 10, 64, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_UNSUPPORTED);
  g.depth_max = 6;
  g.funcs = dup;
  g.n_funcs = 2;
  EXPECT(tgp_generate(&g, 10, 64, o, o + 4096, o + 8192, 64, NULL, NULL), TGP_E_ARG);
  g.funcs = funcs;
  g.n_funcs = 3;
  EXPECT(tgp_generate(&g, 0, 64, NULL, NULL, NULL, 64, NULL, NULL), TGP_OK);
}

static void measurement_calls(void) {
  float* x = (float*)FAKE(9);
  EXPECT(tgp_op_apply(0, x, x, 10, NULL), TGP_E_ARG);
  EXPECT(tgp_op_apply(12, x, x, 10, NULL), TGP_E_ARG);
  EXPECT(tgp_op_apply(7, x, x, -1, NULL), TGP_E_ARG);
  EXPECT(tgp_op_apply(7, NULL, x, 10, NULL), TGP_E_ARG);
  EXPECT(tgp_op_apply(7, NULL, NULL, 0, NULL), TGP_OK);
  EXPECT(tgp_op_cost(12, NULL), TGP_E_ARG);
}

static void status_strings(void) {
  for (int s = -9; s <= 2; ++s) {
    const char* t = tgp_status_str((tgp_status)s);
    if (!t || !*t) {
      fprintf(stderr, "empty status string for %d\n", s);
      g_fail = 1;
    }
  }
}

static void cache_files(const char* dir) {
  char path[4096], saved[4096];
  snprintf(path, sizeof path, "%s/cache.jsonl", dir);
  snprintf(saved, sizeof saved, "%s/saved.jsonl", dir);
  /* two good lines around malformed ones: truncated, overlong (one exactly at the line
   * buffer's size, one far beyond it), bytes outside the architecture alphabet, values out of
   * range, an empty line */
  const char* good1 =
      "{\"arch\":\"gfx950\",\"cus\":256,\"P\":1000,\"Lmax\":64,\"V\":2,\"D\":5000,\"n_out\":1,\"grad\":0,"
      "\"mode\":1,\"block_waves\":4,\"points_per_lane\":8,\"trees_per_unit\":1,\"flags\":0}\n";
  const char* good2 =
      "{\"arch\":\"gfx950\",\"cus\":256,\"P\":7,\"Lmax\":1024,\"V\":16,\"D\":1,\"n_out\":4,\"grad\":1,"
      "\"mode\":2,\"block_waves\":2,\"points_per_lane\":3,\"trees_per_unit\":64,\"flags\":4}\n";
  size_t cap = 1 << 16;
  char* text = (char*)calloc(cap, 1);
  strcat(text, good1);
  strcat(text, "{\"arch\":\"gfx950\",\"cus\":256,\"P\":1000\n");
  size_t n = strlen(text);
  for (int i = 0; i < 511; ++i) text[n++] = 'a';
  text[n++] = '\n';
  for (int i = 0; i < 5000; ++i) text[n++] = '{';
  text[n++] = '\n';
  strcat(text, "{\"arch\":\"gfx\xff\xfe\",\"cus\":256}\n\n");
  strcat(text,
         "{\"arch\":\"gfx950\",\"cus\":256,\"P\":1000,\"Lmax\":64,\"V\":2,\"D\":5000,\"n_out\":1,\"grad\":0,"
         "\"mode\":9,\"block_waves\":4,\"points_per_lane\":8,\"trees_per_unit\":1,\"flags\":0}\n");
  strcat(text,
         "{\"arch\":\"aaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaa\",\"cus\":256,\"P\":1,\"Lmax\":64,"
         "\"V\":2,\"D\":5,\"n_out\":1,\"grad\":0,\"mode\":1,\"block_waves\":4,\"points_per_lane\":8,"
         "\"trees_per_unit\":1,\"flags\":0}\n");
  strcat(text, good2);
  strcat(text, "{");  /* unterminated last line */
  write_file(path, text);
  free(text);
  int32_t ok = -1, bad = -1;
  EXPECT(tgp_autotune_cache_load(path, &ok, &bad), TGP_OK);
  EXPECT(ok, 2);
  EXPECT(bad, 7);
  EXPECT(tgp_autotune_cache_load(path, NULL, NULL), TGP_OK);
  EXPECT(tgp_autotune_cache_save(saved), TGP_OK);
  EXPECT(tgp_autotune_cache_load(saved, &ok, &bad), TGP_OK);
  EXPECT(ok, 2);
  EXPECT(bad, 0);
  EXPECT(tgp_autotune_cache_load(NULL, NULL, NULL), TGP_E_ARG);
  EXPECT(tgp_autotune_cache_save(NULL), TGP_E_ARG);
  snprintf(path, sizeof path, "%s/missing/cache.jsonl", dir);
  EXPECT(tgp_autotune_cache_load(path, NULL, NULL), TGP_E_IO);
  EXPECT(tgp_autotune_cache_save(path), TGP_E_IO);
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s <scratch directory>\n", argv[0]);
    return 2;
  }
  evaluation_calls();
  exchange_and_generation_calls();
  measurement_calls();
  status_strings();
  cache_files(argv[1]);
  if (!g_fail) printf("host checks passed\n");
  return g_fail;
}
