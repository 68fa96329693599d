// Replays a script of C ABI calls (include/lagmean.h) against a library built
// with host sanitizers and linked to the stand-in HIP runtime (hipstub.cpp).
// Test infrastructure only: no result is checked here (no kernel runs), only
// that every call returns the expected status and touches only memory it may.
//
// Script: one operation per line, run ids are small integers.
//   create ID N PREC(0|1) DT INTERP(0|1) FIELDS MODE   lm_create (kin: a plane wave)
//   set ID                lm_set_state from caller buffers freed right after
//   begin ID | step ID K | end ID (then lm_read_mean of every output) | state ID
//   remap ID | peek ID | destroy ID | save ID | restore ID FROM (a checkpoint of run FROM)
//   batch                 a new batch (lm_batch_create); one batch at a time
//   add ID STEPS | remove ID | bstep MAX | btune STEPS REPS | bdestroy | tune ID STEPS REPS
//   expect STATUS         the next call must return STATUS (default LM_OK)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "lagmean.h"

namespace {

std::map<int, lm_run*> runs;
std::map<int, int> sizes;
std::map<int, std::vector<unsigned char>> blobs;  // checkpoints, by the id of the saved run
lm_batch* batch = nullptr;
int expect_next = LM_OK;
long line_no = 0;

void check(lm_status s, const char* what) {
  const int want = expect_next;
  expect_next = LM_OK;
  if (s != want) {
    std::fprintf(stderr, "replay line %ld: %s returned %d (%s: %s), expected %d\n", line_no, what, (int)s,
                 lm_status_str(s), lm_last_error(), want);
    std::exit(3);
  }
}

lm_run* run(int id) {
  auto it = runs.find(id);
  if (it == runs.end()) {
    std::fprintf(stderr, "replay line %ld: unknown run %d\n", line_no, id);
    std::exit(2);
  }
  return it->second;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: replay SCRIPT\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "r");
  if (!f) {
    std::perror(argv[1]);
    return 2;
  }
  char buf[512];
  long ops = 0;
  while (std::fgets(buf, sizeof buf, f)) {
    ++line_no;
    char op[32] = {0};
    if (std::sscanf(buf, "%31s", op) != 1 || op[0] == '#') continue;
    ++ops;
    int id = 0, n = 0, prec = 0, interp = 0, mode = 0, k = 0;
    unsigned fields = 0;
    double dt = 0.0;
    const std::string o = op;
    if (o == "expect") {
      std::sscanf(buf, "%*s %d", &expect_next);
    } else if (o == "create") {
      std::sscanf(buf, "%*s %d %d %d %lf %d %u %d", &id, &n, &prec, &dt, &interp, &fields, &mode);
      lm_config c{};
      c.n = n;
      c.precision = prec;
      c.f = c.g = c.H = 1.0;
      c.dt = dt;
      c.avg_fields = fields;
      c.interp = interp;
      c.mode = mode;
      if (mode == LM_KINEMATIC_PLANEWAVE) {
        c.kin[0] = 2.0;
        c.kin[2] = 0.1;
      }
      lm_run* r = nullptr;
      check(lm_create(&c, nullptr, &r), "lm_create");
      if (r) {
        runs[id] = r;
        sizes[id] = n;
      }
    } else if (o == "set" || o == "state" || o == "peek") {
      std::sscanf(buf, "%*s %d", &id);
      const size_t nn = (size_t)sizes[id] * sizes[id];
      // caller buffers that die right after the call
      std::vector<double>* u = new std::vector<double>(nn, 0.01);
      std::vector<double>* v = new std::vector<double>(nn, -0.02);
      std::vector<double>* h = new std::vector<double>(nn, 1.0);
      if (o == "set") check(lm_set_state(run(id), u->data(), v->data(), h->data(), 0), "lm_set_state");
      else if (o == "state") check(lm_get_state(run(id), u->data(), v->data(), h->data(), 0), "lm_get_state");
      else check(lm_peek(run(id), LM_P_XI_X, u->data(), 0), "lm_peek");
      delete u;
      delete v;
      delete h;
    } else if (o == "begin") {
      std::sscanf(buf, "%*s %d", &id);
      check(lm_begin_interval(run(id)), "lm_begin_interval");
    } else if (o == "step") {
      std::sscanf(buf, "%*s %d %d", &id, &k);
      check(lm_step(run(id), k), "lm_step");
    } else if (o == "end") {
      std::sscanf(buf, "%*s %d", &id);
      double T = 0.0;
      const lm_status s = lm_end_interval(run(id), &T);
      check(s, "lm_end_interval");
      const size_t nn = (size_t)sizes[id] * sizes[id];
      for (int kind = LM_K_S2_MEAN; kind <= LM_K_EULER_MEAN && s == LM_OK; ++kind) {
        std::vector<double>* out = new std::vector<double>(nn);
        check(lm_read_mean(run(id), LM_FIELD_FIRST, kind, out->data(), 0), "lm_read_mean");
        delete out;
      }
    } else if (o == "save") {
      std::sscanf(buf, "%*s %d", &id);
      size_t n = 0;
      check(lm_checkpoint_size(run(id), &n), "lm_checkpoint_size");
      blobs[id].assign(n, 0);
      check(lm_save(run(id), blobs[id].data(), n, 0), "lm_save");
    } else if (o == "restore") {
      int from = 0;
      std::sscanf(buf, "%*s %d %d", &id, &from);
      // a copy that dies right after the call
      std::vector<unsigned char>* b = new std::vector<unsigned char>(blobs[from]);
      check(lm_restore(run(id), b->data(), b->size(), 0), "lm_restore");
      delete b;
    } else if (o == "remap") {
      std::sscanf(buf, "%*s %d", &id);
      double res = 0.0;
      check(lm_remap_s1(run(id), 4, &res), "lm_remap_s1");
    } else if (o == "destroy") {
      std::sscanf(buf, "%*s %d", &id);
      const lm_status s = lm_destroy(run(id));
      check(s, "lm_destroy");
      if (s == LM_OK) runs.erase(id);
    } else if (o == "batch") {
      check(lm_batch_create(nullptr, &batch), "lm_batch_create");
    } else if (o == "add") {
      std::sscanf(buf, "%*s %d %d", &id, &k);
      check(lm_batch_add(batch, run(id), k), "lm_batch_add");
    } else if (o == "remove") {
      std::sscanf(buf, "%*s %d", &id);
      check(lm_batch_remove(batch, run(id)), "lm_batch_remove");
    } else if (o == "bstep") {
      std::sscanf(buf, "%*s %d", &k);
      int32_t active = 0;
      check(lm_batch_step(batch, k, &active), "lm_batch_step");
    } else if (o == "btune") {
      int reps = 1;
      std::sscanf(buf, "%*s %d %d", &k, &reps);
      int32_t tuned = 0;
      check(lm_batch_autotune(batch, k, reps, &tuned), "lm_batch_autotune");
    } else if (o == "tune") {
      int reps = 1;
      std::sscanf(buf, "%*s %d %d %d", &id, &k, &reps);
      lm_schedule best{};
      double ms[16];
      int32_t count = 0;
      check(lm_autotune(run(id), k, reps, &best, ms, 16, &count), "lm_autotune");
    } else if (o == "bdestroy") {
      check(lm_batch_destroy(batch), "lm_batch_destroy");
      batch = nullptr;
    } else {
      std::fprintf(stderr, "replay line %ld: unknown operation %s\n", line_no, op);
      return 2;
    }
  }
  std::fclose(f);
  if (batch) check(lm_batch_destroy(batch), "lm_batch_destroy");
  for (auto& r : runs) check(lm_destroy(r.second), "lm_destroy");
  std::printf("replay: %ld operations ok\n", ops);
  return 0;
}
