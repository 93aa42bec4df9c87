/* Oracle internals.  TEST INFRASTRUCTURE (see oracle.h). */
#ifndef DG_ORACLE_INTERNAL_H
#define DG_ORACLE_INTERNAL_H

#include "oracle.h"

double orc_phi(int dim, const int *e, const double *xi);
double orc_dphi(int dim, const int *e, const double *xi, int axis);
double orc_ref_mass(int dim, const int *e);
double orc_pressure(int dim, double gamma, const double *u);

/* A leaf block: tree index, level (roots are level 1) and its integer
 * position inside the tree at that level. */
typedef struct {
    int tree, level, idx[3];
} orc_key;

/* One piece of a guard cell: the part of the guard cell covered by one
 * source cell.  Boxes are in global integer units (see forest.c). */
typedef struct {
    int leaf;        /* source leaf */
    int cell;        /* source cell inside that leaf */
    long lo[3], hi[3]; /* overlap box, unwrapped to the guard cell's frame */
    long src_lo[3];  /* source cell lower corner in the same frame */
    long src_size;   /* source cell edge */
} orc_piece;

typedef struct {
    int kind;        /* 0 copy (same level), 1 projection, 2 outflow mirror */
    int npiece;
    orc_piece *piece;
} orc_guard_plan;

/* Neighbour relation across one face of a leaf, found geometrically. */
typedef struct {
    int boundary;    /* 1: domain boundary with outflow condition */
    int nn;          /* number of face neighbours (1, or 2^(d-1) when finer) */
    int nb[4];
    int level_diff;  /* neighbour level - own level: -1, 0, +1 */
} orc_face_nbr;

struct orc_forest {
    int dim, p, N, nb, nv, q;
    int roots[3];
    double lo[3], hi[3];
    int bc[3];
    int max_level;
    double gamma;
    int hanging;
    int equation;     /* ORC_EQ_EULER or ORC_EQ_ADVECTION */
    double vel[3];    /* advection velocity */
    double nu;        /* diffusion coefficient */
    double avec[3];   /* exact diffusion solution exp(a . x + nu |a|^2 t) */
    double time;      /* time of the state (Dirichlet data) */
    double stage_time; /* time of the stage input the residual sees */
    long unit;        /* global units per root edge = N * 2^(max_level-1) */
    int nleaves;
    orc_key *leaf;
    int *exps;        /* nb x 3 */
    orc_face_nbr *fn; /* nleaves x 2d */
    orc_guard_plan *gp; /* nleaves x 2d x N^(d-1) */
    int *frame;       /* rotation code of each root's local frame (NULL: all 0) */
    double *nodes;    /* 2-D root grid nodes (x, y) of bilinear roots, (roots_x + 1) x
                         (roots_y + 1), x fastest (NULL: the axis-aligned box grid) */
    /* adaptation plan */
    int new_n;
    orc_key *new_leaf;
};

/* geometry helpers shared by the oracle's own files */
/* frame matrix of a root: global vector = Q * local vector */
void orc_frame_matrix(const orc_forest *f, int tree, int Q[3][3]);
/* global box (lower corner, edge) of a leaf, in global units */
void orc_leaf_box(const orc_forest *f, const orc_key *k, long *lo, long *size);
/* the same in the coordinates of the leaf's own root (local frame, the
 * root's lower corner at 0) */
void orc_leaf_lbox(const orc_forest *f, const orc_key *k, long *lo, long *size);
/* global lower corner of the leaf's cell with local index ijk */
void orc_cell_gbox(const orc_forest *f, const orc_key *k, const int *ijk, long *lo);
long orc_domain_units(const orc_forest *f, int axis);
void orc_build_topology(orc_forest *f);
void orc_free_topology(orc_forest *f);
int orc_ncell(const orc_forest *f);
int orc_nface_cells(const orc_forest *f);
void orc_cell_ijk(const orc_forest *f, int cell, int *ijk);
int orc_cell_index(const orc_forest *f, const int *ijk);
void orc_sort_leaves(const orc_forest *f, orc_key *leaves, int n);
/* find the leaf of the current forest containing global point x (unwrapped
 * coordinates are wrapped on periodic axes); -1 if outside the domain */
int orc_find_leaf(const orc_forest *f, const orc_key *leaves, int n, const double *x);

#endif
