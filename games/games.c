/*
 * Fast builders for the synthetic cooperative games used as inputs by the
 * tests and the benchmark. They construct value vectors from a game's own
 * definition (no part of the FSI operator is computed here):
 *   planted sparse game:  v(S) = sum_k c_k [A_k subset of S]
 *   tree-ensemble game:   v(S) = sum_trees tree(z(S)),
 *                         z(S)_f = x_f if f in S else b_f
 * Bit i of a mask <=> feature i.
 *
 * Build: gcc -O2 -shared -fPIC games.c -o libgames.so
 */
#include <stdint.h>

/* v must be zeroed by the caller (length 2^d). */
void games_planted(double *v, int d, int n_terms, const int64_t *masks,
                   const double *coefs)
{
    const int64_t full = ((int64_t)1 << d) - 1;
    for (int k = 0; k < n_terms; ++k) {
        const int64_t A = masks[k] & full;
        const int64_t comp = full & ~A;
        const double c = coefs[k];
        int64_t sub = 0;
        for (;;) {
            v[A | sub] += c;
            if (sub == comp) break;
            sub = (sub - comp) & comp;
        }
    }
}

/*
 * Full binary trees of the given depth in heap order: internal node i has
 * children 2i+1 (left, z_f < thr) and 2i+2 (right, z_f >= thr); the
 * 2^depth leaves follow the 2^depth - 1 internal nodes.
 * feat/thr: n_trees x (2^depth - 1); leaf: n_trees x 2^depth; x, b: d.
 * For every leaf, the coalitions that reach it form a subcube of the mask
 * space: path features whose test fails at b must be in S, those whose test
 * fails at x must be out of S, all others are free. Every S reaches exactly
 * one leaf per tree, so the work per tree is 2^d. v must be zeroed.
 */
void games_tree(double *v, int d, int n_trees, int depth, const int *feat,
                const double *thr, const double *leaf, const double *x,
                const double *b)
{
    const int n_int = (1 << depth) - 1;
    const int n_leaf = 1 << depth;
    const int64_t full = ((int64_t)1 << d) - 1;
    for (int tr = 0; tr < n_trees; ++tr) {
        const int *F = feat + (int64_t)tr * n_int;
        const double *TH = thr + (int64_t)tr * n_int;
        const double *LV = leaf + (int64_t)tr * n_leaf;
        for (int lf = 0; lf < n_leaf; ++lf) {
            /* okx / okb: features whose tests all pass at x / at b */
            int64_t on_path = 0, failx = 0, failb = 0;
            int node = n_int + lf; /* heap index of the leaf */
            while (node > 0) {
                const int parent = (node - 1) / 2;
                const int right = (node == 2 * parent + 2);
                const int f = F[parent];
                const double t = TH[parent];
                const int px = right ? (x[f] >= t) : (x[f] < t);
                const int pb = right ? (b[f] >= t) : (b[f] < t);
                on_path |= (int64_t)1 << f;
                if (!px) failx |= (int64_t)1 << f;
                if (!pb) failb |= (int64_t)1 << f;
                node = parent;
            }
            if (failx & failb) continue; /* unreachable leaf */
            const int64_t need = failb;   /* must be in S (x passes there) */
            const int64_t forbid = failx; /* must be out of S */
            const int64_t freeb = full & ~(need | forbid);
            const double val = LV[lf];
            int64_t sub = 0;
            for (;;) {
                v[need | sub] += val;
                if (sub == freeb) break;
                sub = (sub - freeb) & freeb;
            }
            (void)on_path;
        }
    }
}
