// Host-side compiler from postfix formula bytecode to the micro-operations the
// census kernels interpret.
//
// Every rewrite below is an exact semantic identity, so the compiled program
// computes the same truth set as the input on every model (Theorem 1):
//   - constant folding: a & TOP = a, a & BOT = BOT, a | TOP = TOP, ...,
//     BOX TOP = TOP, DIA BOT = BOT; DIA TOP and BOX BOT become frame literals;
//   - negation normal form: De Morgan, a -> b = ~a | b, and the modal
//     dualities ~BOX a = DIA ~a, ~DIA a = BOX ~a, ~(a <-> b) = a <-> ~b;
//   - operand order of the (then commutative) binary nodes is chosen by the
//     Sethi-Ullman rule so the stack of saved truth sets stays shallow, and a
//     literal operand is consumed directly instead of being loaded.
#include <algorithm>
#include <vector>
#include <cstdio>

#include "kripke_internal.h"
#include "../../include/kripke.h"

namespace kripke {
namespace {

enum Kind : uint8_t { K_CONST, K_LEAF, K_AND, K_OR, K_IFF, K_BOX, K_DIA };

struct IR {
  Kind kind;
  uint8_t leaf;  // K_CONST: 0/1; K_LEAF: L_* id
  int a, b;
};

struct Builder {
  std::vector<IR> nodes;

  int add(Kind k, uint8_t leaf, int a, int b) {
    nodes.push_back(IR{k, leaf, a, b});
    return (int)nodes.size() - 1;
  }
  bool is_const(int i, int v) const {
    return nodes[i].kind == K_CONST && nodes[i].leaf == v;
  }
  int mk_const(int v) { return add(K_CONST, (uint8_t)v, -1, -1); }
  int mk_leaf(uint8_t l) { return add(K_LEAF, l, -1, -1); }
  int mk_and(int p, int q) {
    if (is_const(p, 0) || is_const(q, 0)) return mk_const(0);
    if (is_const(p, 1)) return q;
    if (is_const(q, 1)) return p;
    return add(K_AND, 0, p, q);
  }
  int mk_or(int p, int q) {
    if (is_const(p, 1) || is_const(q, 1)) return mk_const(1);
    if (is_const(p, 0)) return q;
    if (is_const(q, 0)) return p;
    return add(K_OR, 0, p, q);
  }
  int mk_iff(int p, int q) {
    if (nodes[p].kind == K_CONST) return nodes[p].leaf ? q : negate(q);
    if (nodes[q].kind == K_CONST) return nodes[q].leaf ? p : negate(p);
    return add(K_IFF, 0, p, q);
  }
  int mk_box(int p) {
    if (is_const(p, 1)) return mk_const(1);
    if (is_const(p, 0)) return mk_leaf(L_DEAD);
    return add(K_BOX, 0, p, -1);
  }
  int mk_dia(int p) {
    if (is_const(p, 0)) return mk_const(0);
    if (is_const(p, 1)) return mk_leaf(L_SUCC);
    return add(K_DIA, 0, p, -1);
  }
  // Negation normal form of the negation of node i.
  int negate(int i) {
    IR n = nodes[i];
    switch (n.kind) {
      case K_CONST: return mk_const(!n.leaf);
      case K_LEAF:
        if (n.leaf < 4) return mk_leaf((uint8_t)(L_NVAR0 + n.leaf));
        if (n.leaf < 8) return mk_leaf((uint8_t)(n.leaf - 4));
        if (n.leaf == L_SUCC) return mk_leaf(L_DEAD);
        return mk_leaf(L_SUCC);
      case K_AND: return mk_or(negate(n.a), negate(n.b));
      case K_OR: return mk_and(negate(n.a), negate(n.b));
      case K_IFF: return mk_iff(n.a, negate(n.b));
      case K_BOX: return mk_dia(negate(n.a));
      case K_DIA: return mk_box(negate(n.a));
    }
    return -1;
  }
};

// Parse and validate postfix bytecode into folded NNF IR.  Returns the root.
int build_ir(Builder& B, const uint8_t* code, uint32_t len, uint32_t nvars, std::string* err) {
  if (len == 0 || len > (uint32_t)kMaxProgram) {
    *err = "program length must be 1.." + std::to_string(kMaxProgram);
    return KRIPKE_ELIMIT;
  }
  std::vector<int> st;
  for (uint32_t i = 0; i < len; ++i) {
    uint8_t op = code[i];
    if (op == B_TOP || op == B_BOT) {
      st.push_back(B.mk_const(op == B_TOP));
    } else if (op >= B_VAR0 && op < B_VAR0 + 4) {
      if ((uint32_t)(op - B_VAR0) >= nvars) {
        *err = "variable p_" + std::to_string(op - B_VAR0) + " used with nvars=" +
               std::to_string(nvars);
        return KRIPKE_EPROGRAM;
      }
      st.push_back(B.mk_leaf((uint8_t)(L_VAR0 + op - B_VAR0)));
    } else if (op == B_NOT || op == B_BOX || op == B_DIA) {
      if (st.empty()) {
        *err = "stack underflow at node " + std::to_string(i);
        return KRIPKE_EPROGRAM;
      }
      int a = st.back();
      st.pop_back();
      st.push_back(op == B_NOT ? B.negate(a) : op == B_BOX ? B.mk_box(a) : B.mk_dia(a));
    } else if (op == B_AND || op == B_OR || op == B_IMP || op == B_IFF) {
      if (st.size() < 2) {
        *err = "stack underflow at node " + std::to_string(i);
        return KRIPKE_EPROGRAM;
      }
      int b = st.back();
      st.pop_back();
      int a = st.back();
      st.pop_back();
      int r;
      if (op == B_AND) r = B.mk_and(a, b);
      else if (op == B_OR) r = B.mk_or(a, b);
      else if (op == B_IMP) r = B.mk_or(B.negate(a), b);
      else r = B.mk_iff(a, b);
      st.push_back(r);
    } else {
      *err = "unknown opcode " + std::to_string(op) + " at node " + std::to_string(i);
      return KRIPKE_EPROGRAM;
    }
  }
  if (st.size() != 1) {
    *err = "program leaves " + std::to_string(st.size()) + " values on the stack";
    return KRIPKE_EPROGRAM;
  }
  return st[0];
}

struct Emitter {
  const Builder& B;
  std::vector<int> need;
  Compiled* out;

  bool leaf(int i) const { return B.nodes[i].kind == K_LEAF; }

  int compute_need(int i) {
    const IR& n = B.nodes[i];
    int r = 0;
    switch (n.kind) {
      case K_CONST:
      case K_LEAF: r = 0; break;
      case K_BOX:
      case K_DIA: r = compute_need(n.a); break;
      default: {
        int na = compute_need(n.a), nb = compute_need(n.b);
        if (leaf(n.b)) r = na;
        else if (leaf(n.a)) r = nb;
        else r = std::max(std::max(na, nb), std::min(na, nb) + 1);
      }
    }
    need[i] = r;
    return r;
  }

  void emit(int i, int depth) {
    const IR& n = B.nodes[i];
    std::vector<uint8_t>& m = out->micro;
    switch (n.kind) {
      case K_CONST:
        m.push_back((uint8_t)(U_LOAD + (n.leaf ? L_TOP : L_BOT)));
        out->loads++;
        return;
      case K_LEAF:
        m.push_back((uint8_t)(U_LOAD + n.leaf));
        out->loads++;
        return;
      case K_BOX:
      case K_DIA: {
        // a chain of modal operators over its innermost operand: a literal
        // operand is consumed by the first modal op, the rest go in pairs
        std::vector<int> chain;  // outermost first
        int x = i;
        while (B.nodes[x].kind == K_BOX || B.nodes[x].kind == K_DIA) {
          chain.push_back(B.nodes[x].kind == K_DIA ? 1 : 0);
          x = B.nodes[x].a;
        }
        out->modal += (int)chain.size();
        size_t k = chain.size();  // next modal op to apply is chain[k-1]
        if (leaf(x) && B.nodes[x].leaf < L_SUCC) {
          m.push_back((uint8_t)((chain[k - 1] ? U_DIA_L : U_BOX_L) + B.nodes[x].leaf));
          --k;
        } else {
          emit(x, depth);
        }
        while (k >= 2) {
          m.push_back((uint8_t)(U_MM + 2 * chain[k - 1] + chain[k - 2]));
          k -= 2;
        }
        if (k == 1) m.push_back(chain[0] ? U_DIA : U_BOX);
        return;
      }
      default: break;
    }
    uint8_t base_l = n.kind == K_AND ? U_AND_L : n.kind == K_OR ? U_OR_L : U_IFF_L;
    uint8_t base_s = n.kind == K_AND ? U_AND_S : n.kind == K_OR ? U_OR_S : U_IFF_S;
    out->binary++;
    if (leaf(n.b) || leaf(n.a)) {
      int lf = leaf(n.b) ? n.b : n.a;
      int other = leaf(n.b) ? n.a : n.b;
      emit(other, depth);
      m.push_back((uint8_t)(base_l + B.nodes[lf].leaf));
      return;
    }
    int first = need[n.a] >= need[n.b] ? n.a : n.b;
    int second = first == n.a ? n.b : n.a;
    emit(first, depth);
    m.push_back((uint8_t)(U_SAVE + depth));
    out->saves++;
    emit(second, depth + 1);
    m.push_back((uint8_t)(base_s + depth));
  }
};

int finish(Builder& B, int root, Compiled* out, std::string* err) {
  Emitter E{B, std::vector<int>(B.nodes.size(), 0), out};
  out->micro.clear();
  out->modal = out->binary = out->loads = out->saves = 0;
  out->is_const = B.nodes[root].kind == K_CONST ? B.nodes[root].leaf : -1;
  out->slots = E.compute_need(root);
  if (out->slots > kMaxSlots) {
    *err = "program needs " + std::to_string(out->slots) + " stack slots (max " +
           std::to_string(kMaxSlots) + ")";
    return KRIPKE_ELIMIT;
  }
  E.emit(root, 0);
  out->micro.push_back(U_END);
  return KRIPKE_OK;
}

}  // namespace

int compile_program(const uint8_t* code, uint32_t len, uint32_t nvars, Compiled* out,
                    std::string* err) {
  Builder B;
  B.nodes.reserve(4 * len + 8);
  int root = build_ir(B, code, len, nvars, err);
  if (root < 0) return root;
  return finish(B, root, out, err);
}

int compile_iff(const uint8_t* a, uint32_t la, const uint8_t* b, uint32_t lb, uint32_t nvars,
                Compiled* out, std::string* err) {
  Builder B;
  B.nodes.reserve(4 * (la + lb) + 8);
  int ra = build_ir(B, a, la, nvars, err);
  if (ra < 0) return ra;
  int rb = build_ir(B, b, lb, nvars, err);
  if (rb < 0) return rb;
  return finish(B, B.mk_iff(ra, rb), out, err);
}

}  // namespace kripke
