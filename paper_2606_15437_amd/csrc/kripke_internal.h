// Internal definitions shared by the host program compiler and the kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace kripke {

// Input bytecode (postfix, one byte per node), as documented in kripke.h.
enum : uint8_t {
  B_TOP = 0, B_BOT = 1, B_VAR0 = 2, B_NOT = 6, B_AND = 7, B_OR = 8, B_IMP = 9,
  B_BOX = 10, B_DIA = 11, B_IFF = 12
};

// Leaves of compiled programs.  After constant folding and negation normal
// form, leaves are literals p_i / ~p_i and the frame-only literals
// DIA TOP ("has a successor") and BOX BOT ("dead end"); TOP/BOT survive only
// as whole programs.
enum : uint8_t {
  L_VAR0 = 0,   // p_i        (0..3)
  L_NVAR0 = 4,  // not p_i    (4..7)
  L_SUCC = 8,   // DIA TOP
  L_DEAD = 9,   // BOX BOT
  L_TOP = 10,
  L_BOT = 11,
  L_OPERANDS = 10,  // leaves usable as a binary operand (0..9)
};

// Micro-operations of the accumulator machine the kernels interpret.  ACC
// holds the current truth set (one 32-valuation word per world); SAVE d
// copies ACC to stack slot d, OP_S d combines slot d into ACC.
enum : uint8_t {
  U_END = 0,
  U_LOAD = 1,     // + leaf (0..11): ACC = leaf
  U_AND_L = 13,   // + leaf (0..9):  ACC = ACC & leaf
  U_OR_L = 23,    // + leaf:         ACC = ACC | leaf
  U_IFF_L = 33,   // + leaf:         ACC = ACC <-> leaf
  U_BOX = 43,     // ACC = BOX ACC  (Lemma 1, containment)
  U_DIA = 44,     // ACC = DIA ACC  (Lemma 1, intersection)
  U_SAVE = 45,    // + d (0..7)
  U_AND_S = 53,   // + d: ACC = slot[d] & ACC
  U_OR_S = 61,    // + d
  U_IFF_S = 69,   // + d
  // superinstructions (one dispatch for a common pair)
  U_DIA_L = 77,   // + leaf (0..9): ACC = DIA leaf
  U_BOX_L = 87,   // + leaf (0..9): ACC = BOX leaf
  U_MM = 97,      // + 2*first + second (modal 0 BOX, 1 DIA): ACC = second(first(ACC))
  U_NCODES = 101
};

constexpr int kMaxSlots = 8;
constexpr int kMaxProgram = 255;
constexpr int kMaxMicro = 2 * kMaxProgram + 2;

struct Compiled {
  std::vector<uint8_t> micro;  // terminated by U_END
  int slots = 0;               // stack slots needed
  int modal = 0, binary = 0, loads = 0, saves = 0;  // executed micro-op counts
  int is_const = -1;           // 0/1 if the whole formula folds to BOT/TOP
};

// Validate and compile one program.  Returns 0 or a negative KRIPKE_E* code
// with a message in *err.
int compile_program(const uint8_t* code, uint32_t len, uint32_t nvars, Compiled* out,
                    std::string* err);

// Build the biconditional of two programs and compile it.
int compile_iff(const uint8_t* a, uint32_t la, const uint8_t* b, uint32_t lb, uint32_t nvars,
                Compiled* out, std::string* err);

}  // namespace kripke
