// Host-side forest topology for the block-AMR DG library: leaves of the
// block trees (Sec. 3.1), face links between leaves (same level, coarser,
// finer, domain boundary), refinement planning with 2:1 face balance and
// the inheritance plan of Sec. 3.4.  Keys live in a hash map, so every link
// is an O(1) lookup.
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dgamr.h"

namespace dgamr {

struct Key {
    int tree = 0, level = 1;
    int idx[3] = {0, 0, 0};
};

enum LinkType : int { LINK_SAME = 0, LINK_COARSE = 1, LINK_FINE = 2, LINK_BOUNDARY = 3 };

// Neighbour relation across one face (in the leaf's local frame).
// SAME/COARSE: nbr[0].  FINE: the 2^(d-1) finer leaves, ordered by their
// tangential position (lower axis bit fastest).  COARSE: off[k] is this
// leaf's half (0/1) along the k-th tangential axis inside the coarse
// neighbour's face.  rot: 0 when the neighbour's root has the same frame;
// else 1 + the index of this face's first guard-cell plan (RotPlan), and
// nbr/off are not used by the kernels.
struct FaceLink {
    int type;
    int nbr[4];
    int off[2];
    int rot;
};
static_assert(sizeof(FaceLink) == 32, "FaceLink is uploaded as 8 int32");

// Per-leaf geometry uploaded to the device, along the leaf's local axes.
struct LeafGeo {
    double scale[3]; // 2 / h_a
    double lo[3];    // physical position of the leaf's local origin corner
    double h[3];     // cell edge per local axis
    double vol;      // cell volume
    int level;
    int pad;
    signed char q[12]; // the root's frame Q (q[3 g + l]): global vector = Q local
    // bilinear / trilinear roots (Forest::set_nodes): the leaf's physical
    // corners, corner b at reference coordinate -1 or +1 along axis a by bit
    // a of b; zero otherwise
    double node[8][3];
};

// Guard cell across a face between roots of different frames (Sec. 3.5:
// K_d = R^n K_s, R^n S^i K_s or R^n C(K_s...)): the source cells in the
// neighbour's frame, the operator applied there, and the rotation into the
// destination frame.  m[3 l' + l]: the source's reference coordinate l' is
// m times the destination's coordinate l (a signed permutation); momentum
// goes to the destination frame with its transpose.
enum PlanType : int { PLAN_COPY = 0, PLAN_SPLIT = 1, PLAN_COMBINE = 2 };
struct RotPlan {
    int type;
    int child;       // PLAN_SPLIT: position of the guard cell inside the source cell (source frame)
    int leaf[8];     // COPY/SPLIT: [0]; COMBINE: fine cell of child position c (source frame)
    int cell[8];
    signed char m[12];
};

// frame matrix of a rotation code: 2-D quarter turns counter-clockwise;
// 3-D the code-th signed permutation matrix of determinant +1 (the
// permutations of the local axes in lexicographic order, then the sign
// patterns, bit l = local axis l negative).  Q[g][l]: global = Q local.
void frame_matrix(int dim, int code, int Q[3][3]);

// Inheritance of one new leaf: copied, split from a parent or combined
// from 2^d children of the old forest.
enum InheritType : int { INH_COPY = 0, INH_SPLIT = 1, INH_COMBINE = 2 };
struct Inherit {
    int type;
    int src[8];  // COPY/SPLIT: src[0]; COMBINE: child c (bit a = upper half along a)
    int child;   // SPLIT: this leaf's position inside the parent
};

class Forest {
  public:
    explicit Forest(const dgamr_forest_desc &d);

    // validates the descriptor; returns DGAMR_OK or an error with text
    static int validate(const dgamr_forest_desc &d, std::string &err);

    int dim() const { return desc_.dim; }
    // variables per cell: d + 2 (Euler) or 1 (scalar convection, diffusion)
    int nv() const { return scalar() ? 1 : desc_.dim + 2; }
    bool advection() const { return desc_.equation == DGAMR_EQ_ADVECTION; }
    bool diffusion() const { return desc_.equation == DGAMR_EQ_DIFFUSION; }
    bool scalar() const { return desc_.equation != DGAMR_EQ_EULER; }
    int n() const { return static_cast<int>(leaves_.size()); }
    const std::vector<Key> &leaves() const { return leaves_; }
    const std::vector<FaceLink> &links() const { return links_; }
    const dgamr_forest_desc &desc() const { return desc_; }

    // rebuilds links_ (and the guard plans of rotated faces); DGAMR_EBALANCE
    // on a 2:1 violation
    int build_links(std::string &err);
    // rotation codes of the root frames (one per tree), before any refinement
    int set_frames(const int32_t *codes, std::string &err);
    bool rotated() const { return rotated_; }
    // Sec. 3.3, Eq. 6: roots as bilinear (3-D: trilinear) images of the
    // reference square (cube), from the root grid nodes, x fastest
    int set_nodes(const double *xy, std::string &err);
    bool mapped() const { return !nodes_.empty(); }
    // steps run the guard fill before every stage kernel (the far side is
    // not taken inline) and a CFL reduction per step (none folded into the
    // stages)
    bool unfused() const { return rotated_ || mapped(); }
    const std::vector<RotPlan> &plans() const { return plans_; }
    std::vector<LeafGeo> geometry() const;

    // refinement planning and switching; see dgamr_set_refinement
    int plan(const int8_t *flags, std::string &err);
    bool has_plan() const { return has_plan_; }
    int planned_n() const { return static_cast<int>(planned_.size()); }
    // replaces the leaves by the plan; fills the inheritance list (indexed
    // by new leaf, sources are old leaf ids)
    int commit(std::vector<Inherit> &inh, std::string &err);

  private:
    uint64_t pack(int tree, int level, const int *idx) const;
    int find(int tree, int level, const int *idx) const;
    bool neighbour_root(int tree, int axis, int side, int &out) const;
    uint64_t morton(const Key &k) const;
    void sort_keys(std::vector<Key> &v) const;
    void reindex();

    dgamr_forest_desc desc_;
    std::vector<Key> leaves_;
    std::unordered_map<uint64_t, int> index_;
    std::vector<FaceLink> links_;
    std::vector<int> frame_;      // per tree (empty: all 0)
    bool rotated_ = false;        // some root has a non-zero frame
    std::vector<double> nodes_;   // bilinear root grid nodes (empty: the box grid)
    std::vector<RotPlan> plans_;  // guard-cell plans of rotated faces
    int frame_of(int tree) const { return frame_.empty() ? 0 : frame_[tree]; }
    bool rot_plans(int i, int face, const FaceLink &L);
    std::vector<Key> planned_;
    std::vector<Inherit> planned_inh_;
    bool has_plan_ = false;
};

} // namespace dgamr
