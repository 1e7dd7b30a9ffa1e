// Host-only logic of the library, free of any HIP call: the functor-chain
// compiler (Sec. 3.3, Tab. "functors"), the transfer-table bake, the camera
// basis and the screen rectangle of a job.  Compiled into the library and, on
// its own, into a sanitizer harness that feeds it hostile inputs on the CPU.
#pragma once

#include <string>

#include "isaac_internal.h"

namespace isaac {
namespace host {

struct CompiledChain {
    int n_ops = 0;
    int out_dim = 1;
    DevOp ops[kMaxOps];
};

// Parse "name(args) | name | ..." for an f_dim-component source into at most
// kMaxOps bytecode ops (after exact simplifications); false with a message in
// err on a bad chain.
bool compile_chain(const char* text, int f_dim, CompiledChain& out, std::string& err);

// T[j] = PL(j / 255), j = 0..255, as 4 floats per entry into table (256 x 4);
// false with a message on invalid points (fewer than 2, not spanning [0,1] with
// strictly increasing x, a value outside [0,1] or NaN).
bool bake_tf(const isaac_tf_point* pts, int n, float* table, std::string& err);

struct CameraBasis {
    double fwd[3], right[3], upp[3], h, aspect;
};

// Orthonormal forward/right/up' of a render descriptor's camera and the
// half-height of the view; false with a message for a degenerate camera.
bool camera_basis(const isaac_render_desc& j, CameraBasis& cb, std::string& err);

// A pixel rectangle [cull[0], cull[2]] x [cull[1], cull[3]] of the job's image
// containing every pixel whose ray can meet its box (from the job's camera,
// size, dims and origin); the whole image when a box corner lies at or behind
// the eye plane.
void set_cull_rect(DevJob& dj);

}  // namespace host
}  // namespace isaac
