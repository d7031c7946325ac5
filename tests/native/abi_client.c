/* A plain C99 client of the library's C ABI, host calls only: it builds a
 * 1D stencil graph task by task, compiles it, runs the host models of a list
 * launch and of a gang launch over it (checking the execution order against
 * every edge), and computes the last-user dependences of a three-task
 * implicit program whose DAG is known by hand. */
#include <stdint.h>
#include <stdio.h>

#include "taskgraph.h"

#define CHECK(call)                                                                     \
  do {                                                                                  \
    tg_status s_ = (call);                                                              \
    if (s_ != TG_OK) {                                                                  \
      printf("FAIL %s: status %d (%s)\n", #call, (int)s_, tg_last_error());            \
      return 1;                                                                         \
    }                                                                                   \
  } while (0)
#define EXPECT(cond)                                 \
  do {                                               \
    if (!(cond)) {                                   \
      printf("FAIL %s (line %d)\n", #cond, __LINE__); \
      return 1;                                      \
    }                                                \
  } while (0)

enum { W = 6, T = 5, N = W * T };

int main(void) {
  tg_graph g;
  tg_event ev[N];
  uint32_t pred_lo[N], pred_hi[N];
  CHECK(tg_graph_create(&g, TG_EXPLICIT, 64, 0, 7));
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < W; ++i) {
      tg_event p[3];
      uint32_t np = 0;
      const int lo = i > 0 ? i - 1 : 0, hi = i < W - 1 ? i + 1 : W - 1;
      if (t > 0)
        for (int j = lo; j <= hi; ++j) p[np++] = ev[(t - 1) * W + j];
      CHECK(tg_task_add(g, p, np, 2, &ev[t * W + i]));
      pred_lo[t * W + i] = (uint32_t)lo;
      pred_hi[t * W + i] = (uint32_t)hi;
    }
  CHECK(tg_graph_finalize(g));
  uint64_t n = 0;
  CHECK(tg_graph_num_tasks(g, &n));
  EXPECT(n == N);

  /* list launch model: 3 workers, window 64, default schedule */
  uint64_t order[N], executed = 0, makespan = 0, bound = 0;
  CHECK(tg_emulate_schedule(&g, 1, 3, 64, 0, 11, order, &executed, &makespan, &bound));
  EXPECT(executed == N);
  EXPECT(makespan >= bound && bound > 0);
  uint32_t at[N];
  for (uint32_t k = 0; k < N; ++k) at[k] = 0xFFFFFFFFu;
  for (uint32_t k = 0; k < N; ++k) {
    const uint32_t e = (uint32_t)(order[k] & 0xFFFFFFFFu);
    EXPECT((order[k] >> 32) == 0 && e < N && at[e] == 0xFFFFFFFFu);
    at[e] = k;
  }
  for (int t = 1; t < T; ++t)
    for (int i = 0; i < W; ++i)
      for (uint32_t j = pred_lo[t * W + i]; j <= pred_hi[t * W + i]; ++j)
        EXPECT(at[(t - 1) * W + j] < at[t * W + i]);

  /* gang launch model: 3 gangs of 4 members, every share once */
  uint64_t shares = 0;
  CHECK(tg_emulate_gang(&g, 1, 3, 4, 64, 0, 5, 0, &shares));
  EXPECT(shares == 4u * N);
  CHECK(tg_graph_destroy(g));

  /* last-user dependences: t0 writes [0,4); t1 writes [4,8) and reads [3,4);
   * t2 writes [2,6).  Edges: t0 -> t1 (t1 reads what t0 wrote), t0 -> t2
   * (both write 2..3), t1 -> t2 (t2 overwrites 3, which t1 read, and 4..5,
   * which t1 wrote). */
  const uint64_t req_ptr[4] = {0, 1, 3, 4};
  const tg_region_req reqs[4] = {{0, 4, TG_RW, 0}, {4, 8, TG_RW, 0}, {3, 4, TG_RO, 0}, {2, 6, TG_RW, 0}};
  uint64_t row_ptr[4], e = 0;
  uint32_t col[8];
  CHECK(tg_last_user_dag(3, req_ptr, reqs, row_ptr, col, 8, &e));
  EXPECT(e == 3);
  EXPECT(row_ptr[0] == 0 && row_ptr[1] == 2 && row_ptr[2] == 3 && row_ptr[3] == 3);
  EXPECT(((col[0] == 1 && col[1] == 2) || (col[0] == 2 && col[1] == 1)) && col[2] == 2);

  printf("abi client ok\n");
  return 0;
}
