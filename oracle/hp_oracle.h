/* Plain CPU oracle (test infrastructure only; see hp_oracle.c). */
#ifndef HP_ORACLE_H
#define HP_ORACLE_H
#include <stdint.h>

enum {
    ORC_OK = 0,
    ORC_INVALID_ARG = 1,
    ORC_INDEX_RANGE = 2,
    ORC_NOT_PERMUTATION = 3,
    ORC_DUPLICATE_INDEX = 4,
    ORC_NOT_CANONICAL = 5,
    ORC_SHAPE = 6
};

enum { ORC_OP_SECOND = 0, ORC_OP_PLUS = 1, ORC_OP_REPLACE = 2 };

int orc_check_csr(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col);

int orc_permute(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                const void *val, int vsize, const int32_t *p, const int32_t *q,
                const int64_t *rows, int64_t ns,
                int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need);

int orc_spref(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
              const void *val, int vsize, const int32_t *I, int64_t nI,
              const int32_t *J, int64_t nJ, const int64_t *rows, int64_t ns,
              int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need);

int orc_spref_dcsc(int64_t m, int64_t n, int64_t nzc, const int32_t *jc, const int64_t *colptr,
                   const int32_t *row, const void *val, int vsize, const int32_t *I, int64_t nI,
                   const int32_t *J, int64_t nJ, const int64_t *cols, int64_t ns,
                   int64_t *out_ptr, int32_t *out_row, void *out_val, int64_t cap, int64_t *need);

int orc_permute_map(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                    const void *val, int vsize, const int32_t *p, const int32_t *q,
                    const int64_t *rows, int64_t ns,
                    int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
                    int nthreads);

int orc_spref_map(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                  const void *val, int vsize, const int32_t *I, int64_t nI,
                  const int32_t *J, int64_t nJ, const int64_t *rows, int64_t ns,
                  int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
                  int nthreads);

int orc_spasgn(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col, const void *val,
               int vsize, int64_t bm, int64_t bn, const int64_t *browptr, const int32_t *bcol,
               const void *bval, const int32_t *I, int64_t nI, const int32_t *J, int64_t nJ,
               int op, const int64_t *rows, int64_t ns,
               int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
               int nthreads);
#endif
