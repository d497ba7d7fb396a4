/*
 * gc_oracle.h -- declarations of the plain CPU oracle (test infrastructure
 * only; see gc_oracle.c).  Not included by any product source.
 */
#ifndef GC_ORACLE_H
#define GC_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#define OR_VERSION 1

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOSPC (-2)
#define OR_ECORRUPT (-3)
#define OR_ENOMEM (-6)

enum { OR_SIMPLE = 0, OR_SCHEME = 1, OR_AFOR = 2, OR_PFD = 3, OR_VSE = 4 };
enum { OR_LD_BINARY = 0, OR_LD_CU = 1, OR_LD_IU = 2 };
enum { OR_PFD_LINKED = 0, OR_PFD_BITMAP = 1 };

typedef struct {
    int codec;     /* OR_SIMPLE .. OR_PFD                            */
    int k;         /* layout width: 4 (the paper) .. 64, power of 2   */
    int cg;        /* Group-Scheme compression granularity 1,2,4,8    */
    int ld;        /* Group-Scheme length descriptor                  */
    int delta;     /* input is docIDs: code d-gaps, decode prefix sum */
    int pfd_pos;   /* Group-PFD exception positions: linked / bitmap  */
    int zeta_num;  /* Group-PFD exception-ratio threshold num/den     */
    int zeta_den;
} or_params;

int or_bw(uint32_t x);
void or_tuple_max(const uint32_t *x, size_t T, int k, uint32_t *qmax);
void or_dgap(const uint32_t *d, size_t n, uint32_t *g);
void or_prefix_sum(const uint32_t *g, size_t n, uint32_t *d);
void or_gsim_table(int *num, int *bw);
size_t or_gsim_select(const uint32_t *MaxArr, size_t L, uint8_t *ModeArr);
int or_parse_header(uint32_t w0, or_params *p);
int or_gsc_units(uint32_t quadmax, int cg);
size_t or_afor_partition(const uint32_t *qmax, size_t M, int k, uint8_t *Fout);
size_t or_vse_partition(const uint32_t *qmax, size_t M, int k, uint8_t *Fout);
int or_pfd_width(const uint32_t *qmax, int ntuples, int num, int den);
long or_encode(const uint32_t *in, size_t n, const or_params *p, uint32_t *out, size_t cap);
long or_gsim_encode_with(const uint32_t *in, size_t n, const or_params *p, const uint8_t *sel,
                         size_t S, uint32_t *out, size_t cap);
long or_afor_encode_with(const uint32_t *in, size_t n, const or_params *p, const uint8_t *F,
                         size_t nf, uint32_t *out, size_t cap);
long or_decode(const uint32_t *s, size_t words, uint32_t *out, size_t cap);

/* per-block container of the learned selector (see gc_oracle.c) */
#define OR_BLOCK_INTS 128
#define OR_NCLASS 16
int or_block_class_params(int kappa, or_params *p);
long or_block_encode(const uint32_t *x, int kappa, uint32_t *payload, size_t cap, uint32_t *blockword);
long or_block_size(const uint32_t *x, int kappa);
int or_block_best(const uint32_t *x, long *sizes);
int or_block_decode(uint32_t blockword, const uint32_t *payload, size_t words, uint32_t *x);
void or_block_features(const uint32_t *x, double *f);
long or_blockmix_encode(const uint32_t *in, size_t n, const uint8_t *kappas, uint32_t *out, size_t cap,
                        uint8_t *kappa_out);
long or_blockmix_decode(const uint32_t *s, size_t words, uint32_t *out, size_t cap);

#endif
