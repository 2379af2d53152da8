/* oracle_internal.h -- private helpers of the oracle (test infrastructure). */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include <stddef.h>
#include "oracle.h"

void og_set_error(const char* msg);

/* padded grid: two ghost layers in each used direction */
typedef struct {
  int dim, n[3], P[3], o[3];
  size_t npad, ncell;
} og_pad;

void og_pad_init(og_pad* pd, const og_grid* g);
static inline size_t og_pidx(const og_pad* pd, int i, int j, int k)
{
  return (size_t)(i + pd->o[0]) + (size_t)pd->P[0] * ((size_t)(j + pd->o[1]) + (size_t)pd->P[1] * (size_t)(k + pd->o[2]));
}
static inline size_t og_cidx(const og_pad* pd, int i, int j, int k)
{
  return (size_t)i + (size_t)pd->n[0] * ((size_t)j + (size_t)pd->n[1] * (size_t)k);
}
#endif
