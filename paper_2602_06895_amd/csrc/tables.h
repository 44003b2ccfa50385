// Device-resident channel and process tables.
//
// The host channel compiler turns each diagram topology into one ChannelTab:
// the time-like invariants with their bounds written as linear forms over the
// square roots of earlier invariants (the min/max mass recursion of the
// s-channel integration order, and the t-channel bounds, resolved once at
// construction), the chain of 2->2 blocks, the (phi, theta) decays and the
// momentum slot of every particle.  Every lane of a wave runs the same
// channel, so kernels read these tables with scalar loads and index the
// per-event register file with wave-uniform slot numbers.
//
// Slots are tied to the operation that writes them, so every write has an
// index known at compile time: 2->2 block b writes slots 2b, 2b + 1 from the
// bottom; decay d writes slots NS - 2 - 2d, NS - 1 - 2d from the top of an
// NS-slot file.  A slot code c >= 0 names bottom slot c, c < 0 names top
// slot NS + c, so the tables do not depend on the kernel's NS.
#pragma once

#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

namespace msx {

constexpr int kMaxFinal = 8;        // final-state particles per process
constexpr int kMaxInv = 8;          // s-hat plus time-like invariants per channel
constexpr int kMaxSlots = 2 * (kMaxFinal - 1);  // momentum slots per event
constexpr int kMaxDims = 32;        // random dimensions per channel
constexpr int kMaxUniq = 16;        // distinct propagator invariants per process
constexpr int kMaxChanPerProc = 32; // channels per process (local weights)
constexpr int kMaxFactors = 8;      // integrand propagator factors
constexpr int kMaxChannels = 64;    // channels per context
constexpr int kMaxProcesses = 8;
constexpr int kMaxBins = 128;       // VEGAS bins per dimension

enum MapKind : int32_t {
    MAP_FIXED = 0,  // value fixed (lepton beams: s-hat = s)
    MAP_FLAT = 1,   // nu = 0
    MAP_POW = 2,    // power law, nu != 0, 1
    MAP_LOG = 3,    // nu = 1
    MAP_BW = 4,     // Breit-Wigner
    MAP_RAMBO = 5   // FastRambo cluster mass (int_pow = k, e = 1/k, mw = c_k)
};

// Parameters of one G_nu / G_BW mapping.
struct MapParams {
    int32_t kind;
    int32_t int_pow;  // MAP_POW: 1/(1-nu) when it is a small integer, else 0
    double m2;        // pole: m^2, or -a for a massless structure; BW: m^2
    double mw;        // BW: m * Gamma
    double e;         // MAP_POW: 1 - nu
    double inv_e;     // MAP_POW: 1 / (1 - nu)
};

// Source of a mass: sqrt of invariant `inv` when inv >= 0, else the constant.
struct MassSrc {
    int32_t inv;
    int32_t pad;
    double m;
};

// One time-like invariant.  Index 0 is s-hat with static bounds.  Others:
//   m_min = min_const + sum_{j in min_mask} sqrt(s_j)
//   m_max = sqrt(s_parent) - max_const - sum_{j in max_mask} sqrt(s_j)
struct InvSpec {
    MapParams map;
    int32_t parent;
    uint32_t min_mask;
    uint32_t max_mask;
    uint32_t set;  // final-state particles whose momenta sum to the invariant's cluster
    double min_const, max_const;
    // static bounds (s-hat): precomputed A = (xmax - m2)^e, B = (xmin - m2)^e
    // (MAP_POW), logs (MAP_LOG) or arctangents u2, u1 (MAP_BW)
    double xmin, xmax, A, B;
};

// One 2->2 block of the t-channel chain (section 2.2.4).
struct BlockSpec {
    MassSrc m1, m2;
    MapParams tmap;  // |t| mapping: G_nu with the massless auxiliary pole
    int32_t side;    // 0: p1 is a leg next to A (p_A -= p1); 1: p2 is a leg next
                     // to B (p_B -= p2); 2: last block (both outputs are legs)
    int32_t com;     // p_A, p_B are the incoming partons in their CM frame
    int32_t m0_inv;  // (p_A + p_B)^2 = s[m0_inv] (s-hat or the previous t-channel invariant)
    uint32_t set1, set2;  // final-state particles making up the outputs p1, p2
};

// One (phi, theta) two-body decay (section 2.2.3).
struct DecaySpec {
    int32_t parent_rest;  // 1: parent at rest in the partonic frame (no boost)
    int32_t parent_slot;  // slot code of the parent momentum otherwise
    int32_t parent_inv;   // m0^2 = s[parent_inv]
    uint32_t parent_set;  // final-state particles of the parent
    MassSrc m1, m2;
    uint32_t set1, set2;  // final-state particles of the first two children
    int32_t kind;         // 0 two-body; 1 three-body (its third child takes the
                          // first slot of the next entry); 2 that next entry
    uint32_t set3;        // three-body: final-state particles of the third child
    MassSrc m3;
};

struct ChannelTab {
    int32_t process;
    int32_t dims;
    int32_t n_final;
    int32_t n_inv;       // including s-hat
    int32_t n_blocks;
    int32_t n_decays;
    int32_t hadronic;
    int32_t alpha_index; // position of this channel within its process
    int32_t n_slots;     // 2 (n_blocks + n_decays) = 2 (n_final - 1)
    int32_t kinds;       // map kinds used (bitmask, see chain.h)
    double jac_const;    // (2 pi)^(4 - 3 n) times the channel constant
    InvSpec inv[kMaxInv];
    BlockSpec blk[kMaxFinal];
    DecaySpec dec[kMaxFinal];
    int32_t final_slot[kMaxFinal];  // slot code of each final-state particle
    int32_t st;                     // 1: blocks after the first use (s~, t) (section 2.2.5)
    // Chili channels (no tree): particle k sits in slot k
    int32_t chili;                  // 1: a Chili channel
    double chili_ptmin2;            // the process's p_T cut squared (<= 0: none)
    double chili_m[kMaxFinal];      // final-state masses
};

// Integrand and local channel weights of one process.
// Everything the integrand needs about one distinct invariant, read with
// one scalar load per invariant.
struct UniqSpec {
    uint32_t set;    // particle set
    int32_t t;       // 1: q = p_a - sum over the set, 0: q = sum
    int32_t fkind;   // integrand factor on q^2: 0 none, 1 Breit-Wigner, 2 1/(|q^2| + mu^2)
    int32_t massive; // channel-weight form: 1 massive, 0 massless, -1 not in any channel
    double fa, fb;   // factor constants: (m^2, (m w)^2) or (mu^2, 0)
    double am2, amw2;  // channel-weight constants (m^2, (m w)^2)
};

struct ProcessTab {
    int32_t n_final;
    int32_t hadronic;
    int32_t n_chan;      // channels entering alpha (1: alpha = 1)
    int32_t n_uniq;      // distinct invariants q^2 needed
    int32_t n_fprop;     // integrand propagator factors
    int32_t pdf;         // toy PDF on both momentum fractions
    int32_t ang;         // -1, or particle index for 1 + cos^2 theta
    int32_t pdf_b_int;   // pdf_b when it is an integer 1..16, else 0
    double s_lab;
    double pdf_a, pdf_b;
    double pt_min2;      // <= 0: no cut
    double alpha_mu2;
    // distinct invariants: q = p_a - sum (t) or sum (s) over a particle set
    int32_t uniq_t[kMaxUniq];
    uint32_t uniq_set[kMaxUniq];
    // form of each invariant in alpha: massive -> 1/((q^2-m^2)^2 + m^2 w^2),
    // massless -> 1/(|q^2| + mu^2)^2
    int32_t uniq_massive[kMaxUniq];
    double uniq_m2[kMaxUniq];
    double uniq_mw[kMaxUniq];
    uint32_t chan_mask[kMaxChanPerProc];  // invariants of each channel
    int32_t uniq_f[kMaxUniq];             // integrand factor on each invariant, -1: none
    // integrand factors
    int32_t f_uniq[kMaxFactors];
    int32_t f_bw[kMaxFactors];
    double f_m2[kMaxFactors];
    double f_mw[kMaxFactors];
    double f_mu2[kMaxFactors];
    UniqSpec uq[kMaxUniq];                // the fields above, per invariant
    // channels without a diagram (Chili): constant local weight prior_share;
    // the diagram channels share tree_share by their propagator products
    uint32_t chan_prior;
    int32_t pad_prior;
    double prior_share, tree_share;
};

// Per-call description of a multichannel launch (passed by value).
struct SampleCall {
    int32_t n_chan;
    int32_t ept;                           // events per thread per tile
    int64_t n_tiles;
    uint64_t skip_mask;                    // channels whose events another launch writes (no tiles, no statistics)
    int64_t tile_start[kMaxChannels + 1];  // first tile of each channel
    int64_t ev_start[kMaxChannels + 1];    // first output position
};

}  // namespace msx
