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

// Neighbour relation across one face.  SAME/COARSE: nbr[0].  FINE: the
// 2^(d-1) finer leaves, ordered by their tangential position (lower axis
// bit fastest).  COARSE: off[k] is this leaf's half (0/1) along the k-th
// tangential axis inside the coarse neighbour's face.
struct FaceLink {
    int type;
    int nbr[4];
    int off[2];
    int pad;
};
static_assert(sizeof(FaceLink) == 32, "FaceLink is uploaded as 8 int32");

// Per-leaf geometry uploaded to the device.
struct LeafGeo {
    double scale[3]; // 2 / h_a
    double lo[3];    // physical lower corner of the leaf
    double h[3];     // cell edge per axis
    double vol;      // cell volume
    int level;
    int pad;
};

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

    // rebuilds links_; DGAMR_EBALANCE on a 2:1 violation
    int build_links(std::string &err);
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
    std::vector<Key> planned_;
    std::vector<Inherit> planned_inh_;
    bool has_plan_ = false;
};

} // namespace dgamr
