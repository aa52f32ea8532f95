/*
 * mrip_from_c -- the MRIP library driven from plain C through include/mrip.h
 * (no Python, no torch): create a context, run replications on the null
 * stream, read every scalar output back to host memory and its interval.
 *
 *   mrip_from_c pi  <points> <reps> <seed> <mapping>
 *   mrip_from_c mm1 <lambda> <mu> <customers> <reps> <seed> <mapping> [split]
 *   mrip_from_c rw  <walkers> <grid> <steps> <reps> <seed> <mapping> [walker_sites]
 *
 * mapping: simt, wave or lane0. Prints, for every scalar output k, a line
 * "out k v_0 v_1 ..." (int32 outputs as integers, fp32 ones with 9
 * significant digits, which identify the float) and a line
 * "stats k n mean var half_width t_quantile" (fp64, 17 digits). Exits 1
 * with the library's message on any error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mrip.h"

static mrip_ctx g_ctx;

static void check(mrip_status st, const char *what) {
  if (st == MRIP_OK) return;
  fprintf(stderr, "%s: %s (%s)\n", what, mrip_status_string(st),
          g_ctx ? mrip_last_error(g_ctx) : "");
  exit(1);
}

static mrip_mapping parse_mapping(const char *s) {
  if (!strcmp(s, "simt")) return MRIP_MAP_SIMT;
  if (!strcmp(s, "wave")) return MRIP_MAP_WAVE;
  if (!strcmp(s, "lane0")) return MRIP_MAP_LANE0;
  fprintf(stderr, "unknown mapping %s\n", s);
  exit(2);
}

/* Print output k of the last run (n values) and its statistics. */
static void print_output(uint32_t k, uint64_t n, int is_float) {
  void *buf = malloc(n * 4);
  if (!buf) exit(1);
  check(mrip_outputs(g_ctx, k, buf, n * 4, 0), "mrip_outputs");
  printf("out %u", k);
  for (uint64_t i = 0; i < n; ++i) {
    if (is_float)
      printf(" %.9g", (double)((const float *)buf)[i]);
    else
      printf(" %d", ((const int32_t *)buf)[i]);
  }
  printf("\n");
  free(buf);
  mrip_stats_t s;
  check(mrip_stats(g_ctx, k, 0.95, &s), "mrip_stats");
  printf("stats %u %llu %.17g %.17g %.17g %.17g\n", k, (unsigned long long)s.n, s.mean, s.var,
         s.half_width, s.t_quantile);
}

int main(int argc, char **argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: see the header of mrip_from_c.c\n");
    return 2;
  }
  const char *model = argv[1];
  uint64_t reps, seed;
  if (!strcmp(model, "pi") && argc == 6) {
    mrip_pi_params p = {sizeof p, strtoull(argv[2], NULL, 10)};
    reps = strtoull(argv[3], NULL, 10);
    seed = strtoull(argv[4], NULL, 10);
    check(mrip_create(&g_ctx, MRIP_PI, &p, parse_mapping(argv[5])), "mrip_create");
    check(mrip_run(g_ctx, reps, seed, NULL), "mrip_run");
    print_output(0, reps, 0);
    print_output(1, reps, 1);
  } else if (!strcmp(model, "mm1") && (argc == 8 || argc == 9)) {
    mrip_mm1_params p = {sizeof p, strtof(argv[2], NULL), strtof(argv[3], NULL),
                         strtoull(argv[4], NULL, 10), 0};
    reps = strtoull(argv[5], NULL, 10);
    seed = strtoull(argv[6], NULL, 10);
    check(mrip_create(&g_ctx, MRIP_MM1, &p, parse_mapping(argv[7])), "mrip_create");
    if (argc == 9) check(mrip_set_split(g_ctx, (uint32_t)strtoul(argv[8], NULL, 10)), "split");
    check(mrip_run(g_ctx, reps, seed, NULL), "mrip_run");
    for (uint32_t k = 0; k < 3; ++k) print_output(k, reps, 1);
  } else if (!strcmp(model, "rw") && (argc == 8 || argc == 9)) {
    const uint32_t sites = argc == 9 ? (uint32_t)strtoul(argv[8], NULL, 10) : 0u;
    mrip_rw_params p = {sizeof p, (uint32_t)strtoul(argv[2], NULL, 10),
                        (uint32_t)strtoul(argv[3], NULL, 10),
                        (uint32_t)strtoul(argv[4], NULL, 10), sites};
    reps = strtoull(argv[5], NULL, 10);
    seed = strtoull(argv[6], NULL, 10);
    check(mrip_create(&g_ctx, MRIP_RW, &p, parse_mapping(argv[7])), "mrip_create");
    check(mrip_run(g_ctx, reps, seed, NULL), "mrip_run");
    for (uint32_t k = 0; k < (sites ? 3u : 2u); ++k) print_output(k, reps, 0);
  } else {
    fprintf(stderr, "bad arguments\n");
    return 2;
  }
  mrip_destroy(g_ctx);
  return 0;
}
