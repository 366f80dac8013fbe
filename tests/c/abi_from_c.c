/* A plain C99 client of the library: the header compiles as C, the library
 * links, and calls that fail their host-side argument checks return the
 * documented status and message without touching a GPU. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lor.h"

static int fails = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAIL: %s (last error: %s)\n", what, lor_last_error());
    ++fails;
  }
}

int main(void) {
  lor_sched s;
  int64_t nnz = 0;
  const int32_t* fake = (const int32_t*)(uintptr_t)0x1000; /* never dereferenced */
  expect(lor_abi_version() == 3, "ABI version 3");
  expect(lor_sched_bytes() == sizeof(lor_sched), "schedule size agrees with the header");
  memset(&s, 0, sizeof s);
  expect(lor_pattern(LOR_H1, 0, 1, 8, fake, (int32_t*)fake, &nnz, NULL, &s, NULL) == LOR_EINVAL, "p = 0 rejected");
  expect(strstr(lor_last_error(), "p = 0") != NULL, "message names p");
  expect(lor_pattern(LOR_H1, 6, (int64_t)1 << 30, 8, fake, (int32_t*)fake, &nnz, NULL, &s, NULL) == LOR_EOVERFLOW,
         "index overflow rejected");
  expect(lor_assemble_h1(2, 1, 27, 0, fake, NULL, NULL, 1.0, fake, &s, NULL, LOR_F64, 0u, 10.0, NULL, NULL) ==
             LOR_EINVAL,
         "batch 0 rejected");
  expect(lor_backward_workspace(0, 1, 1, LOR_F64) == 0, "no workspace for an invalid degree");
  expect(lor_backward_workspace(2, 1, 1, LOR_F32) == 8 * 3 * 27, "workspace of one p = 2 element");
  expect(lor_pattern_workspace(LOR_H1, 2, 1, 27) > 0, "schedule bytes of one element");
  printf("%s\n", fails ? "abi_from_c: failures" : "abi_from_c: ok");
  return fails ? 1 : 0;
}
