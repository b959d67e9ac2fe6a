// Scalar expressions on the device (Section 3.2.1): a postfix program over
// device scalars is compiled once on the host (Eval) into a short register
// program -- repeated subexpressions shared, correctly rounded subexpressions
// of constants folded, only IEEE-exact rewrites -- and executed by one
// single-workgroup kernel per call (Execute), however many operations and
// outputs (MultiEval) it has.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "internal.h"

namespace apcg {
namespace {

constexpr int kMaxTokens = 256;
constexpr int kMaxInstr = 128;
constexpr int kMaxIO = 16;

// One register instruction: dst = op(a, b) or a load; registers live in LDS.
struct Instr {
    int16_t op;   // APCG_EXPR_* (INPUT: load input `a`; CONST: load imm)
    int16_t dst;
    int16_t a, b;
    double imm;
};

struct ExecArgs {
    Instr code[kMaxInstr];
    int32_t ncode;
    int32_t nout;
    int16_t out_reg[kMaxIO];
    const double *in[kMaxIO];
    double *out[kMaxIO];
};

bool is_unary(int op) { return op >= APCG_EXPR_NEG && op <= APCG_EXPR_COS; }
bool is_binary(int op) { return op >= APCG_EXPR_ADD && op <= APCG_EXPR_MAX; }
bool is_exact(int op) { return op != APCG_EXPR_EXP && op != APCG_EXPR_LOG && op != APCG_EXPR_SIN && op != APCG_EXPR_COS; }

__host__ __device__ double apply(int op, double a, double b) {
    switch (op) {
        case APCG_EXPR_NEG: return -a;
        case APCG_EXPR_RECIP: return 1.0 / a;
        case APCG_EXPR_SQRT: return sqrt(a);
        case APCG_EXPR_ABS: return fabs(a);
        case APCG_EXPR_EXP: return exp(a);
        case APCG_EXPR_LOG: return log(a);
        case APCG_EXPR_SIN: return sin(a);
        case APCG_EXPR_COS: return cos(a);
        case APCG_EXPR_ADD: return a + b;
        case APCG_EXPR_SUB: return a - b;
        case APCG_EXPR_MUL: return a * b;
        case APCG_EXPR_DIV: return a / b;
        case APCG_EXPR_MIN: return fmin(a, b);
        case APCG_EXPR_MAX: return fmax(a, b);
        default: return 0.0;
    }
}

// Thread 0 runs the program; registers in LDS.
__global__ __launch_bounds__(64) void k_expr(ExecArgs args) {
    __shared__ double reg[kMaxInstr];
    if (threadIdx.x != 0) return;
    for (int i = 0; i < args.ncode; ++i) {
        const Instr &c = args.code[i];
        double v;
        if (c.op == APCG_EXPR_INPUT) v = *args.in[c.a];
        else if (c.op == APCG_EXPR_CONST) v = c.imm;
        else v = apply(c.op, reg[c.a], c.b >= 0 ? reg[c.b] : 0.0);
        reg[c.dst] = v;
    }
    for (int o = 0; o < args.nout; ++o) *args.out[o] = reg[args.out_reg[o]];
}

// DAG node of the compiled expression (hash-consed: equal nodes are one).
struct Node {
    int op;
    int a, b;        // child nodes (-1: none); INPUT: a = input index
    uint64_t bits;   // CONST: the value's bits
    double value;
};

}  // namespace
}  // namespace apcg

struct apcg_expr_s {
    std::vector<apcg::Instr> code;
    std::vector<int16_t> out_reg;
    int32_t ninputs = 0, noutputs = 0;
    int32_t folded = 0, shared = 0;
};

using namespace apcg;

extern "C" {

apcg_status apcg_expr_compile(const apcg_expr_token *prog, int32_t ntokens, int32_t ninputs, int32_t noutputs,
                              apcg_expr *out) {
    try {
        if (!prog || !out || ntokens < 1 || ntokens > kMaxTokens)
            return set_error(APCG_ERR_INVALID_ARG, "expression: bad program size");
        if (ninputs < 0 || ninputs > kMaxIO || noutputs < 1 || noutputs > kMaxIO)
            return set_error(APCG_ERR_INVALID_ARG, "expression: 0..16 inputs and 1..16 outputs");
        std::vector<Node> nodes;
        std::map<std::tuple<int, int, int, uint64_t>, int> memo;
        int32_t folded = 0, shared = 0;
        auto make = [&](int op, int a, int b, double value) -> int {
            uint64_t bits = 0;
            if (op == APCG_EXPR_CONST) memcpy(&bits, &value, sizeof bits);
            const auto key = std::make_tuple(op, a, b, bits);
            auto it = memo.find(key);
            if (it != memo.end()) {
                if (op != APCG_EXPR_INPUT && op != APCG_EXPR_CONST) ++shared;
                return it->second;
            }
            nodes.push_back(Node{op, a, b, bits, value});
            memo[key] = (int)nodes.size() - 1;
            return (int)nodes.size() - 1;
        };
        auto is_const = [&](int k, double v) {
            if (nodes[k].op != APCG_EXPR_CONST) return false;
            uint64_t bits;
            memcpy(&bits, &v, sizeof bits);
            return nodes[k].bits == bits;  // the exact value, sign of zero included
        };
        std::vector<int> stack, outputs(noutputs, -1);
        for (int t = 0; t < ntokens; ++t) {
            const apcg_expr_token &tk = prog[t];
            if (tk.op == APCG_EXPR_INPUT) {
                if (tk.arg < 0 || tk.arg >= ninputs) return set_error(APCG_ERR_INVALID_ARG, "expression: input index");
                stack.push_back(make(APCG_EXPR_INPUT, tk.arg, -1, 0.0));
            } else if (tk.op == APCG_EXPR_CONST) {
                stack.push_back(make(APCG_EXPR_CONST, -1, -1, tk.value));
            } else if (is_unary(tk.op)) {
                if (stack.empty()) return set_error(APCG_ERR_INVALID_ARG, "expression: stack underflow");
                const int a = stack.back();
                stack.pop_back();
                int r;
                if (nodes[a].op == APCG_EXPR_CONST && is_exact(tk.op)) {
                    ++folded;
                    r = make(APCG_EXPR_CONST, -1, -1, apply(tk.op, nodes[a].value, 0.0));
                } else if (tk.op == APCG_EXPR_NEG && nodes[a].op == APCG_EXPR_NEG) {
                    r = nodes[a].a;  // -(-x) = x
                } else {
                    r = make(tk.op, a, -1, 0.0);
                }
                stack.push_back(r);
            } else if (is_binary(tk.op)) {
                if (stack.size() < 2) return set_error(APCG_ERR_INVALID_ARG, "expression: stack underflow");
                const int b = stack.back();
                stack.pop_back();
                const int a = stack.back();
                stack.pop_back();
                int r;
                if (nodes[a].op == APCG_EXPR_CONST && nodes[b].op == APCG_EXPR_CONST) {
                    ++folded;
                    r = make(APCG_EXPR_CONST, -1, -1, apply(tk.op, nodes[a].value, nodes[b].value));
                } else if ((tk.op == APCG_EXPR_MUL && is_const(b, 1.0)) || (tk.op == APCG_EXPR_DIV && is_const(b, 1.0)) ||
                           (tk.op == APCG_EXPR_SUB && is_const(b, 0.0)) || (tk.op == APCG_EXPR_ADD && is_const(b, -0.0))) {
                    r = a;
                } else if ((tk.op == APCG_EXPR_MUL && is_const(a, 1.0)) || (tk.op == APCG_EXPR_ADD && is_const(a, -0.0))) {
                    r = b;
                } else {
                    r = make(tk.op, a, b, 0.0);
                }
                stack.push_back(r);
            } else if (tk.op == APCG_EXPR_OUTPUT) {
                if (tk.arg < 0 || tk.arg >= noutputs) return set_error(APCG_ERR_INVALID_ARG, "expression: output index");
                if (outputs[tk.arg] >= 0) return set_error(APCG_ERR_INVALID_ARG, "expression: output written twice");
                if (stack.empty()) return set_error(APCG_ERR_INVALID_ARG, "expression: stack underflow");
                outputs[tk.arg] = stack.back();
                stack.pop_back();
            } else {
                return set_error(APCG_ERR_INVALID_ARG, "expression: unknown token");
            }
        }
        if (!stack.empty()) return set_error(APCG_ERR_INVALID_ARG, "expression: values left on the stack");
        for (int o = 0; o < noutputs; ++o)
            if (outputs[o] < 0) return set_error(APCG_ERR_INVALID_ARG, "expression: output not written");
        // emit the nodes the outputs reach, children first (node order is
        // already topological: a node is created after its children)
        std::vector<char> live(nodes.size(), 0);
        for (int o : outputs) live[o] = 1;
        for (int k = (int)nodes.size() - 1; k >= 0; --k)
            if (live[k] && nodes[k].op != APCG_EXPR_INPUT && nodes[k].op != APCG_EXPR_CONST) {
                if (nodes[k].a >= 0) live[nodes[k].a] = 1;
                if (nodes[k].b >= 0) live[nodes[k].b] = 1;
            }
        std::vector<int> reg_of(nodes.size(), -1);
        apcg_expr e = new apcg_expr_s();
        for (size_t k = 0; k < nodes.size(); ++k) {
            if (!live[k]) continue;
            if ((int)e->code.size() >= kMaxInstr) {
                delete e;
                return set_error(APCG_ERR_INVALID_ARG, "expression: more than 128 instructions");
            }
            const Node &nd = nodes[k];
            Instr in{};
            in.op = (int16_t)nd.op;
            in.dst = (int16_t)e->code.size();
            in.a = -1;
            in.b = -1;
            if (nd.op == APCG_EXPR_INPUT) in.a = (int16_t)nd.a;
            else if (nd.op == APCG_EXPR_CONST) in.imm = nd.value;
            else {
                in.a = (int16_t)reg_of[nd.a];
                in.b = nd.b >= 0 ? (int16_t)reg_of[nd.b] : (int16_t)-1;
            }
            reg_of[k] = in.dst;
            e->code.push_back(in);
        }
        for (int o : outputs) e->out_reg.push_back((int16_t)reg_of[o]);
        e->ninputs = ninputs;
        e->noutputs = noutputs;
        e->folded = folded;
        e->shared = shared;
        *out = e;
        return APCG_SUCCESS;
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_expr_stats(apcg_expr e, int32_t *instructions, int32_t *folded, int32_t *shared) {
    if (!e) return set_error(APCG_ERR_INVALID_ARG, "expression is NULL");
    if (instructions) *instructions = (int32_t)e->code.size();
    if (folded) *folded = e->folded;
    if (shared) *shared = e->shared;
    return APCG_SUCCESS;
}

apcg_status apcg_expr_execute(apcg_expr e, apcg_ctx ctx, const apcg_scalar *inputs, const apcg_scalar *outputs) {
    try {
        if (!e || !ctx || !outputs || (e->ninputs > 0 && !inputs))
            return set_error(APCG_ERR_INVALID_ARG, "NULL argument");
        ExecArgs args;
        memset(&args, 0, sizeof args);
        std::vector<Acc> acc;
        for (int i = 0; i < e->ninputs; ++i) {
            if (!inputs[i] || inputs[i]->device != ctx->device)
                return set_error(APCG_ERR_INVALID_ARG, "expression input missing or on another device");
            args.in[i] = inputs[i]->d;
        }
        for (int o = 0; o < e->noutputs; ++o) {
            if (!outputs[o] || outputs[o]->device != ctx->device)
                return set_error(APCG_ERR_INVALID_ARG, "expression output missing or on another device");
            for (int q = 0; q < o; ++q)
                if (outputs[q] == outputs[o]) return set_error(APCG_ERR_INVALID_ARG, "expression output repeated");
            args.out[o] = outputs[o]->d;
            args.out_reg[o] = e->out_reg[o];
        }
        // every input read, every output written (a scalar both: read-write)
        for (int i = 0; i < e->ninputs; ++i) {
            bool seen = false;
            for (auto &a : acc)
                if (a.rec == &inputs[i]->rec) seen = true;
            if (!seen) acc.push_back(Acc{&inputs[i]->rec, ACC_R});
        }
        for (int o = 0; o < e->noutputs; ++o) {
            bool seen = false;
            for (auto &a : acc)
                if (a.rec == &outputs[o]->rec) {
                    a.mode = ACC_RW;
                    seen = true;
                }
            if (!seen) acc.push_back(Acc{&outputs[o]->rec, ACC_W});
        }
        args.ncode = (int32_t)e->code.size();
        args.nout = e->noutputs;
        for (int i = 0; i < args.ncode; ++i) args.code[i] = e->code[i];
        apcg_status s;
        if ((s = op_begin(ctx, acc.data(), (int)acc.size()))) return s;
        hipLaunchKernelGGL(k_expr, dim3(1), dim3(64), 0, ctx->stream, args);
        APCG_CHECK_LAUNCH("k_expr");
        return op_end(ctx, acc.data(), (int)acc.size());
    } catch (const std::bad_alloc &) {
        return set_error(APCG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

apcg_status apcg_expr_destroy(apcg_expr e) {
    if (!e) return set_error(APCG_ERR_INVALID_ARG, "expression is NULL");
    delete e;
    return APCG_SUCCESS;
}

}  // extern "C"
