// System description: parser, validation and derived quantities (host).
//
// The text is the ProtoBuf text form of the paper's Appendix A:
//   substeps, dt, gravity{x y z}, bodies{...}, joints{...}, actuators{...}
// extended with the quantities the paper leaves to the engine: colliders
// (sphere, capsule, box), joint frames (rotation, child_rotation, Euler X-Y-Z
// in degrees), spring and damper constants, contact constants (baumgarte,
// elasticity, friction) and the reset clearance.
//
// Readings: DOF = number of angle_limit entries (Appendix A); angles in the
// file are degrees; a body without `inertia` gets that of uniform solid
// colliders; angular_stiffness and limit_stiffness default to stiffness;
// child_rotation defaults to rotation.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../include/braxmi.h"
#include "bx_internal.h"

namespace bx {
namespace {

// ------------------------------------------------------------ tokens
struct Tok {
  enum Kind { ID, STR, NUM, LBRACE, RBRACE, COLON, END } kind;
  std::string text;
  double num = 0;
  int line = 0, col = 0;
};

struct PErr {
  int line, col;
  std::string msg;
};

std::vector<Tok> tokenize(const char* s) {
  std::vector<Tok> out;
  int line = 1, col = 1;
  size_t i = 0, n = std::strlen(s);
  auto adv = [&](size_t k) {
    for (size_t j = 0; j < k; ++j) {
      if (s[i] == '\n') {
        ++line;
        col = 1;
      } else {
        ++col;
      }
      ++i;
    }
  };
  while (i < n) {
    char c = s[i];
    if (c == '#') {
      while (i < n && s[i] != '\n') adv(1);
      continue;
    }
    if (std::isspace((unsigned char)c)) {
      adv(1);
      continue;
    }
    Tok t;
    t.line = line;
    t.col = col;
    if (std::isalpha((unsigned char)c) || c == '_') {
      size_t j = i;
      while (j < n && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
      t.kind = Tok::ID;
      t.text.assign(s + i, j - i);
      adv(j - i);
    } else if (c == '"') {
      size_t j = i + 1;
      while (j < n && s[j] != '"') {
        if (s[j] == '\n') throw PErr{line, col, "unterminated string"};
        ++j;
      }
      if (j >= n) throw PErr{line, col, "unterminated string"};
      t.kind = Tok::STR;
      t.text.assign(s + i + 1, j - i - 1);
      adv(j - i + 1);
    } else if (std::isdigit((unsigned char)c) || c == '-' || c == '+' || c == '.') {
      char* end = nullptr;
      double v = std::strtod(s + i, &end);
      if (end == s + i) throw PErr{line, col, "bad number"};
      t.kind = Tok::NUM;
      t.num = v;
      t.text.assign(s + i, end - (s + i));
      adv((size_t)(end - (s + i)));
    } else if (c == '{') {
      t.kind = Tok::LBRACE;
      adv(1);
    } else if (c == '}') {
      t.kind = Tok::RBRACE;
      adv(1);
    } else if (c == ':') {
      t.kind = Tok::COLON;
      adv(1);
    } else {
      throw PErr{line, col, std::string("unexpected character '") + c + "'"};
    }
    out.push_back(t);
  }
  Tok e;
  e.kind = Tok::END;
  e.line = line;
  e.col = col;
  out.push_back(e);
  return out;
}

// ------------------------------------------------------------ message tree
struct Msg;
struct Val {
  bool is_msg = false;
  Tok tok;                    // scalar value (number, string or identifier)
  std::shared_ptr<Msg> msg;   // nested message
  int line = 0, col = 0;
};
struct Msg {
  std::vector<std::pair<std::string, Val>> fields;
  int line = 0, col = 0;
};

struct Parser {
  std::vector<Tok> t;
  size_t i = 0;
  std::shared_ptr<Msg> message(bool nested) {
    auto m = std::make_shared<Msg>();
    m->line = t[i].line;
    m->col = t[i].col;
    for (;;) {
      const Tok& k = t[i];
      if (k.kind == Tok::END) {
        if (nested) throw PErr{k.line, k.col, "missing '}'"};
        return m;
      }
      if (k.kind == Tok::RBRACE) {
        if (!nested) throw PErr{k.line, k.col, "unbalanced '}'"};
        ++i;
        return m;
      }
      if (k.kind != Tok::ID) throw PErr{k.line, k.col, "expected a field name"};
      std::string name = k.text;
      Val v;
      v.line = k.line;
      v.col = k.col;
      ++i;
      if (t[i].kind == Tok::COLON) {
        ++i;
        if (t[i].kind == Tok::LBRACE) {
          ++i;
          v.is_msg = true;
          v.msg = message(true);
        } else if (t[i].kind == Tok::NUM || t[i].kind == Tok::STR || t[i].kind == Tok::ID) {
          v.tok = t[i];
          ++i;
        } else {
          throw PErr{t[i].line, t[i].col, "expected a value after ':'"};
        }
      } else if (t[i].kind == Tok::LBRACE) {
        ++i;
        v.is_msg = true;
        v.msg = message(true);
      } else {
        throw PErr{t[i].line, t[i].col, "expected ':' or '{' after " + name};
      }
      m->fields.emplace_back(name, v);
    }
  }
};

// ------------------------------------------------------------ field access
struct View {
  const Msg* m;
  void check(const std::set<std::string>& known) const {
    for (auto& f : m->fields)
      if (!known.count(f.first)) throw PErr{f.second.line, f.second.col, "unknown field '" + f.first + "'"};
  }
  const Val* last(const char* name) const {
    const Val* r = nullptr;
    for (auto& f : m->fields)
      if (f.first == name) r = &f.second;
    return r;
  }
  std::vector<const Val*> all(const char* name) const {
    std::vector<const Val*> r;
    for (auto& f : m->fields)
      if (f.first == name) r.push_back(&f.second);
    return r;
  }
  bool has(const char* name) const { return last(name) != nullptr; }
  double num(const char* name, double dflt) const {
    const Val* v = last(name);
    if (!v) return dflt;
    if (v->is_msg || v->tok.kind != Tok::NUM) throw PErr{v->line, v->col, std::string(name) + " must be a number"};
    return v->tok.num;
  }
  std::string str(const char* name) const {
    const Val* v = last(name);
    if (!v) return "";
    if (v->is_msg || v->tok.kind == Tok::NUM) throw PErr{v->line, v->col, std::string(name) + " must be a string"};
    return v->tok.text;
  }
  View sub(const Val* v) const {
    if (!v->is_msg) throw PErr{v->line, v->col, "expected a message"};
    return View{v->msg.get()};
  }
  bool vec(const char* name, double out[3]) const {
    out[0] = out[1] = out[2] = 0;
    const Val* v = last(name);
    if (!v) return false;
    View s = sub(v);
    s.check({"x", "y", "z"});
    out[0] = s.num("x", 0);
    out[1] = s.num("y", 0);
    out[2] = s.num("z", 0);
    return true;
  }
};

struct MErr {
  std::string msg;
};

// ------------------------------------------------------------ geometry
void euler_deg(const double a[3], double R[9]) {
  const double d = M_PI / 180.0;
  double ca = std::cos(a[0] * d), sa = std::sin(a[0] * d), cb = std::cos(a[1] * d), sb = std::sin(a[1] * d);
  double cc = std::cos(a[2] * d), sc = std::sin(a[2] * d);
  // Rx(a) Ry(b) Rz(c)
  R[0] = cb * cc;                 R[1] = -cb * sc;                R[2] = sb;
  R[3] = sa * sb * cc + ca * sc;  R[4] = -sa * sb * sc + ca * cc; R[5] = -sa * cb;
  R[6] = -ca * sb * cc + sa * sc; R[7] = ca * sb * sc + sa * cc;  R[8] = ca * cb;
}

double volume(const ColliderD& c) {
  if (c.kind == 0) return 4.0 / 3.0 * M_PI * c.radius * c.radius * c.radius;
  if (c.kind == 2) return 8.0 * c.half[0] * c.half[1] * c.half[2];
  return M_PI * c.radius * c.radius * (c.length - 2 * c.radius) + 4.0 / 3.0 * M_PI * c.radius * c.radius * c.radius;
}

// principal moments about the collider centre in the collider frame
void principal(const ColliderD& c, double m, double I[3]) {
  if (c.kind == 0) {
    I[0] = I[1] = I[2] = 0.4 * m * c.radius * c.radius;
  } else if (c.kind == 2) {
    double a = c.half[0], b = c.half[1], z = c.half[2];
    I[0] = m * (b * b + z * z) / 3;
    I[1] = m * (a * a + z * z) / 3;
    I[2] = m * (a * a + b * b) / 3;
  } else {
    double r = c.radius, H = c.length - 2 * r;
    double vc = M_PI * r * r * H, vs = 4.0 / 3.0 * M_PI * r * r * r;
    double mc = m * vc / (vc + vs), ms = m - mc;
    I[2] = mc * r * r / 2 + ms * 2 * r * r / 5;
    I[0] = I[1] = mc * (H * H / 12 + r * r / 4) + ms * (2 * r * r / 5 + H * H / 4 + 3 * H * r / 8);
  }
}

}  // namespace

int build_system(const char* text, SystemDesc& d, std::string& err) {
  try {
    Parser p;
    p.t = tokenize(text);
    auto root = p.message(false);
    View top{root.get()};
    top.check({"substeps", "dt", "gravity", "bodies", "joints", "actuators", "baumgarte", "elasticity", "friction",
               "clearance", "body_contacts"});
    d = SystemDesc();
    double sub = top.num("substeps", 1);
    d.dt = top.num("dt", 0.01);
    top.vec("gravity", d.g);
    d.beta = top.num("baumgarte", 0.2);
    d.elasticity = top.num("elasticity", 0.0);
    d.mu = top.num("friction", 1.0);
    d.clearance = top.num("clearance", 0.01);
    if (sub < 1 || sub != std::floor(sub) || sub > 1000) throw MErr{"substeps must be an integer in 1..1000"};
    d.substeps = (int)sub;
    if (!(d.dt > 0)) throw MErr{"dt must be > 0"};
    if (d.mu < 0 || d.beta < 0 || d.elasticity < 0) throw MErr{"friction, baumgarte and elasticity must be >= 0"};

    std::map<std::string, int> bidx;
    for (const Val* bv : top.all("bodies")) {
      View b = top.sub(bv);
      b.check({"name", "mass", "inertia", "frozen", "colliders", "position"});
      BodyD B{};
      B.name = b.str("name");
      if (B.name.empty()) throw MErr{"a body has no name (line " + std::to_string(bv->line) + ")"};
      if (bidx.count(B.name)) throw MErr{"body '" + B.name + "' is defined twice"};
      B.mass = b.num("mass", 0);
      if (!(B.mass > 0)) throw MErr{"body '" + B.name + "': mass must be > 0"};
      for (const Val* cv : b.all("colliders")) {
        View c = b.sub(cv);
        c.check({"position", "rotation", "sphere", "capsule", "box"});
        ColliderD C{};
        c.vec("position", C.pos);
        double rot[3];
        c.vec("rotation", rot);
        euler_deg(rot, C.R);
        int shapes = c.has("sphere") + c.has("capsule") + c.has("box");
        if (shapes != 1) throw MErr{"body '" + B.name + "': a collider needs exactly one shape"};
        if (c.has("sphere")) {
          View s = c.sub(c.last("sphere"));
          s.check({"radius"});
          C.kind = 0;
          C.radius = s.num("radius", 0);
          if (!(C.radius > 0)) throw MErr{"body '" + B.name + "': sphere radius must be > 0"};
        } else if (c.has("capsule")) {
          View s = c.sub(c.last("capsule"));
          s.check({"radius", "length"});
          C.kind = 1;
          C.radius = s.num("radius", 0);
          C.length = s.num("length", 0);
          if (!(C.radius > 0)) throw MErr{"body '" + B.name + "': capsule radius must be > 0"};
          if (C.length < 2 * C.radius) throw MErr{"body '" + B.name + "': capsule length < 2 radius"};
        } else {
          View s = c.sub(c.last("box"));
          s.check({"halfsize"});
          C.kind = 2;
          s.vec("halfsize", C.half);
          if (!(C.half[0] > 0 && C.half[1] > 0 && C.half[2] > 0))
            throw MErr{"body '" + B.name + "': box halfsize must be > 0"};
        }
        B.cols.push_back(C);
      }
      if (b.has("frozen")) {
        View f = b.sub(b.last("frozen"));
        f.check({"position", "rotation"});
        double fp[3], fr[3];
        f.vec("position", fp);
        f.vec("rotation", fr);
        for (int k = 0; k < 3; ++k) {
          B.free_p[k] = fp[k] != 0 ? 0.0 : 1.0;
          B.free_r[k] = fr[k] != 0 ? 0.0 : 1.0;
        }
      } else {
        for (int k = 0; k < 3; ++k) B.free_p[k] = B.free_r[k] = 1.0;
      }
      B.has_pos = b.vec("position", B.pos);
      if (b.has("inertia")) {
        b.vec("inertia", B.I);
      } else {
        if (B.cols.empty()) throw MErr{"body '" + B.name + "': no inertia and no colliders to derive it from"};
        double vol = 0;
        for (auto& C : B.cols) vol += volume(C);
        double I[9] = {0};
        for (auto& C : B.cols) {
          double mc = B.mass * volume(C) / vol, Ip[3];
          principal(C, mc, Ip);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              double v = 0;
              for (int k = 0; k < 3; ++k) v += C.R[3 * i + k] * Ip[k] * C.R[3 * j + k];
              double dd = C.pos[0] * C.pos[0] + C.pos[1] * C.pos[1] + C.pos[2] * C.pos[2];
              v += mc * ((i == j ? dd : 0.0) - C.pos[i] * C.pos[j]);
              I[3 * i + j] += v;
            }
        }
        double dmax = std::max(std::fabs(I[0]), std::max(std::fabs(I[4]), std::fabs(I[8])));
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            if (i != j && std::fabs(I[3 * i + j]) > 1e-9 * dmax)
              throw MErr{"body '" + B.name + "': derived inertia is not diagonal in the body frame; give inertia"};
        B.I[0] = I[0];
        B.I[1] = I[4];
        B.I[2] = I[8];
      }
      if (!(B.I[0] > 0 && B.I[1] > 0 && B.I[2] > 0)) throw MErr{"body '" + B.name + "': inertia must be > 0"};
      bidx[B.name] = (int)d.bodies.size();
      d.bodies.push_back(B);
    }
    if (d.bodies.empty()) throw MErr{"no bodies"};
    if ((int)d.bodies.size() > MAXB) throw MErr{"more than 16 bodies"};

    std::map<std::string, int> jidx;
    std::vector<int> parent_of(d.bodies.size(), -1);
    for (const Val* jv : top.all("joints")) {
      View j = top.sub(jv);
      j.check({"name", "parent", "child", "stiffness", "damping", "angular_stiffness", "angular_damping",
               "limit_stiffness", "parent_offset", "child_offset", "rotation", "child_rotation", "angle_limit"});
      JointD J{};
      J.name = j.str("name");
      std::string pn = j.str("parent"), cn = j.str("child");
      if (!bidx.count(pn)) throw MErr{"joint '" + J.name + "': unknown parent body '" + pn + "'"};
      if (!bidx.count(cn)) throw MErr{"joint '" + J.name + "': unknown child body '" + cn + "'"};
      J.parent = bidx[pn];
      J.child = bidx[cn];
      if (J.parent == J.child) throw MErr{"joint '" + J.name + "': parent and child are the same body"};
      if (parent_of[J.child] >= 0) throw MErr{"joint '" + J.name + "': body '" + cn + "' has two parents"};
      parent_of[J.child] = J.parent;
      if (jidx.count(J.name)) throw MErr{"joint '" + J.name + "' is defined twice"};
      J.k_lin = j.num("stiffness", 0);
      J.c_lin = j.num("damping", 0);
      J.k_ang = j.num("angular_stiffness", J.k_lin);
      J.c_ang = j.num("angular_damping", 0);
      J.k_lim = j.num("limit_stiffness", J.k_lin);
      j.vec("parent_offset", J.ap);
      j.vec("child_offset", J.ac);
      double rot[3], crot[3];
      j.vec("rotation", rot);
      if (!j.vec("child_rotation", crot))
        for (int k = 0; k < 3; ++k) crot[k] = rot[k];
      euler_deg(rot, J.FP);
      euler_deg(crot, J.FC);
      auto lims = j.all("angle_limit");
      if (lims.size() < 1 || lims.size() > 3)
        throw MErr{"joint '" + J.name + "': needs 1 to 3 angle_limit entries (its degrees of freedom)"};
      J.dof = (int)lims.size();
      for (int k = 0; k < J.dof; ++k) {
        View l = j.sub(lims[k]);
        l.check({"min", "max"});
        J.lo[k] = l.num("min", 0) * M_PI / 180.0;
        J.hi[k] = l.num("max", 0) * M_PI / 180.0;
        if (J.lo[k] > J.hi[k]) throw MErr{"joint '" + J.name + "': angle_limit min > max"};
      }
      jidx[J.name] = (int)d.joints.size();
      d.joints.push_back(J);
    }
    if ((int)d.joints.size() > MAXJ) throw MErr{"more than 16 joints"};
    // every body's parent chain must end at a root
    for (size_t b = 0; b < d.bodies.size(); ++b) {
      int x = (int)b, hops = 0;
      while (parent_of[x] >= 0) {
        x = parent_of[x];
        if (++hops > (int)d.bodies.size()) throw MErr{"joints form a cycle"};
      }
    }
    std::vector<int> nch(d.bodies.size(), 0);
    for (auto& J : d.joints)
      if (++nch[J.parent] > MAXCH) throw MErr{"a body has more than 8 children"};

    d.ndof = 0;
    for (auto& J : d.joints) d.ndof += J.dof;
    std::set<int> actuated;
    for (const Val* av : top.all("actuators")) {
      View a = top.sub(av);
      a.check({"name", "joint", "strength", "torque", "angle"});
      std::string jn = a.str("joint");
      if (!jidx.count(jn)) throw MErr{"actuator '" + a.str("name") + "': unknown joint '" + jn + "'"};
      int j = jidx[jn];
      if (actuated.count(j)) throw MErr{"joint '" + jn + "' has two actuators"};
      actuated.insert(j);
      double gear = a.num("strength", 0);
      if (a.has("torque") && a.has("angle"))
        throw MErr{"actuator '" + a.str("name") + "': both torque and angle"};
      const int mode = a.has("angle") ? 1 : 0;
      for (int k = 0; k < d.joints[j].dof; ++k) d.actions.push_back(ActD{j, k, gear, mode});
    }
    if ((int)d.actions.size() > MAXA) throw MErr{"more than 48 actions"};

    for (size_t b = 0; b < d.bodies.size(); ++b) {
      for (auto& C : d.bodies[b].cols) {
        auto add = [&](double x, double y, double z, double rho) {
          ContactD c;
          c.body = (int)b;
          for (int i = 0; i < 3; ++i) c.l[i] = C.pos[i] + C.R[3 * i] * x + C.R[3 * i + 1] * y + C.R[3 * i + 2] * z;
          c.rho = rho;
          d.contacts.push_back(c);
        };
        if (C.kind == 0) {
          add(0, 0, 0, C.radius);
        } else if (C.kind == 1) {
          double hh = C.length / 2 - C.radius;
          add(0, 0, hh, C.radius);
          add(0, 0, -hh, C.radius);
        } else {
          for (int sx = 1; sx >= -1; sx -= 2)
            for (int sy = 1; sy >= -1; sy -= 2)
              for (int sz = 1; sz >= -1; sz -= 2) add(sx * C.half[0], sy * C.half[1], sz * C.half[2], 0.0);
        }
      }
    }
    if ((int)d.contacts.size() > MAXC) throw MErr{"more than 96 contact candidates"};

    // body-body contacts (Section 7.2): every collider of the first body of a
    // declared pair against every collider of the second; each collider is
    // reduced to a core feature plus a radius: a sphere to its centre, a
    // capsule to its axis segment, a box to itself (radius 0). A capsule
    // against a box becomes its two end spheres and its axis segment (the
    // latter a candidate only where its point nearest the box lies strictly
    // between the ends); box against box is not modelled.
    std::vector<int> involved(d.bodies.size(), 0);
    for (const Val* pv : top.all("body_contacts")) {
      View pm = top.sub(pv);
      pm.check({"first", "second"});
      const std::string fa = pm.str("first"), fb = pm.str("second");
      if (!bidx.count(fa) || !bidx.count(fb) || fa == fb)
        throw MErr{"body_contacts: bad pair '" + fa + "' / '" + fb + "'"};
      const int a = bidx[fa], b = bidx[fb];
      for (const ColliderD& ca : d.bodies[a].cols)
        for (const ColliderD& cb : d.bodies[b].cols) {
          if (ca.kind == 2 && cb.kind == 2)
            throw MErr{"body_contacts '" + fa + "' / '" + fb + "': box against box is not modelled"};
          // the segment ends (or the centre) of a sphere or capsule, in its body's frame
          auto ends = [](const ColliderD& c, double e0[3], double e1[3]) {
            const double hh = c.kind == 1 ? c.length / 2 - c.radius : 0.0;
            for (int i = 0; i < 3; ++i) {
              e0[i] = c.pos[i] + c.R[3 * i + 2] * hh;
              e1[i] = c.pos[i] - c.R[3 * i + 2] * hh;
            }
          };
          PairD P{};
          P.a = a;
          P.b = b;
          for (int i = 0; i < 9; ++i) P.aR[i] = P.bR[i] = (i % 4 == 0) ? 1.0 : 0.0;
          if (ca.kind != 2 && cb.kind != 2) {
            ends(ca, P.a0, P.a1);
            ends(cb, P.b0, P.b1);
            P.ra = ca.radius;
            P.rb = cb.radius;
            P.kind = (ca.kind == 1 ? 2 : 0) + (cb.kind == 1 ? 1 : 0);  // PP, PS, SP, SS
            d.pairs.push_back(P);
            continue;
          }
          // one side a box: one candidate per end point of the other side
          const bool box_b = cb.kind == 2;
          const ColliderD& pc = box_b ? ca : cb;
          const ColliderD& bc = box_b ? cb : ca;
          double e[2][3];
          ends(pc, e[0], e[1]);
          const int n_pts = pc.kind == 1 ? 2 : 1;
          for (int k = 0; k < n_pts; ++k) {
            PairD Q = P;
            Q.kind = box_b ? PK_PB : PK_BP;
            double* pt0 = box_b ? Q.a0 : Q.b0;
            double* pt1 = box_b ? Q.a1 : Q.b1;
            double* bx0 = box_b ? Q.b0 : Q.a0;
            double* bx1 = box_b ? Q.b1 : Q.a1;
            double* bh = box_b ? Q.bh : Q.ah;
            double* bR = box_b ? Q.bR : Q.aR;
            for (int i = 0; i < 3; ++i) {
              pt0[i] = pt1[i] = e[k][i];
              bx0[i] = bx1[i] = bc.pos[i];
              bh[i] = bc.half[i];
            }
            for (int i = 0; i < 9; ++i) bR[i] = bc.R[i];
            (box_b ? Q.ra : Q.rb) = pc.radius;
            (box_b ? Q.rb : Q.ra) = 0.0;
            d.pairs.push_back(Q);
          }
          if (pc.kind == 1) {
            // and the capsule's axis segment, a candidate where its point
            // nearest the box lies strictly between the two ends
            PairD Q = P;
            Q.kind = box_b ? PK_SB : PK_BS;
            double* s0 = box_b ? Q.a0 : Q.b0;
            double* s1 = box_b ? Q.a1 : Q.b1;
            double* bx0 = box_b ? Q.b0 : Q.a0;
            double* bx1 = box_b ? Q.b1 : Q.a1;
            double* bh = box_b ? Q.bh : Q.ah;
            double* bR = box_b ? Q.bR : Q.aR;
            for (int i = 0; i < 3; ++i) {
              s0[i] = e[0][i];
              s1[i] = e[1][i];
              bx0[i] = bx1[i] = bc.pos[i];
              bh[i] = bc.half[i];
            }
            for (int i = 0; i < 9; ++i) bR[i] = bc.R[i];
            (box_b ? Q.ra : Q.rb) = pc.radius;
            (box_b ? Q.rb : Q.ra) = 0.0;
            d.pairs.push_back(Q);
          }
        }
    }
    if ((int)d.pairs.size() > MAXP) throw MErr{"more than 32 body-body contact candidates"};
    for (const PairD& P : d.pairs) {
      ++involved[P.a];
      ++involved[P.b];
    }
    for (size_t b = 0; b < d.bodies.size(); ++b)
      if (involved[b] > MAXPI)
        throw MErr{"body '" + d.bodies[b].name + "': more than 16 body-body contact candidates"};
    // each candidate is evaluated on the lane of some body of the system
    // (its handler): the body that evaluates the fewest so far (the lowest
    // index on a tie) among those where the candidate fits, so that the
    // candidates spread over all lanes of an environment. A lane evaluates at
    // most MAXH candidates; in one evaluation slot a body collects at most
    // MAXR shares as a first body and MAXR as a second body.
    const int nb = (int)d.bodies.size();
    std::vector<int> handled(nb, 0);
    std::vector<std::vector<int>> col_a(nb, std::vector<int>(MAXH, 0)), col_b(nb, std::vector<int>(MAXH, 0));
    for (PairD& P : d.pairs) {
      int h = -1;
      for (int want = 0; want < MAXH && h < 0; ++want)
        for (int x = 0; x < nb && h < 0; ++x)
          if (handled[x] == want && col_a[P.a][want] < MAXR && col_b[P.b][want] < MAXR) h = x;
      if (h < 0)
        throw MErr{"body_contacts: bodies '" + d.bodies[P.a].name + "' and '" + d.bodies[P.b].name +
                   "' take part in more candidates than the lanes can evaluate or collect (limit)"};
      P.handler = h;
      const int slot = handled[h]++;
      ++col_a[P.a][slot];
      ++col_b[P.b][slot];
    }
    return BRAX_OK;
  } catch (const PErr& e) {
    err = std::to_string(e.line) + ":" + std::to_string(e.col) + ": " + e.msg;
    return BRAX_E_PARSE;
  } catch (const MErr& e) {
    err = e.msg;
    return BRAX_E_MODEL;
  }
}

void pack_type(const SystemDesc& d, Tables& tab, int t) {
  TypeT& ty = tab.type[t];
  ty = TypeT{};
  ty.nb = (int)d.bodies.size();
  ty.nj = (int)d.joints.size();
  ty.nc = (int)d.contacts.size();
  ty.na = (int)d.actions.size();
  ty.ndof = d.ndof;
  ty.substeps = d.substeps;
  ty.dt = (float)d.dt;
  const double h = d.dt / d.substeps;
  ty.h = (float)h;
  ty.beta_h = (float)(d.beta / h);
  ty.one_plus_e = (float)(1.0 + d.elasticity);
  ty.mu = (float)d.mu;
  ty.clearance = (float)d.clearance;
  for (int k = 0; k < 3; ++k) ty.g[k] = (float)d.g[k];
  ty.frozen = 0;
  for (const BodyD& bd : d.bodies)
    for (int k = 0; k < 3; ++k)
      if (bd.free_p[k] == 0 || bd.free_r[k] == 0) ty.frozen = 1;

  std::vector<int> joint_of(ty.nb, -1);
  for (int j = 0; j < ty.nj; ++j) joint_of[d.joints[j].child] = j;
  for (int b = 0; b < ty.nb; ++b) {
    const BodyD& S = d.bodies[b];
    BodyT& B = tab.body[t][b];
    B = BodyT{};
    B.m = (float)S.mass;
    B.inv_m = (float)(1.0 / S.mass);
    for (int k = 0; k < 3; ++k) {
      B.I[k] = (float)S.I[k];
      B.Iinv[k] = (float)(1.0 / S.I[k]);
      B.free_p[k] = (float)S.free_p[k];
      B.free_r[k] = (float)S.free_r[k];
      B.pos0[k] = (float)S.pos[k];
    }
    B.has_pos = S.has_pos ? 1 : 0;
    B.joint = joint_of[b];
    B.parent = B.joint >= 0 ? d.joints[B.joint].parent : -1;
    B.c0 = B.c1 = 0;
    B.nch = 0;
  }
  for (int j = 0; j < ty.nj; ++j) {
    BodyT& P = tab.body[t][d.joints[j].parent];
    P.ch_packed |= (uint32_t)d.joints[j].child << (4 * P.nch);
    P.ch[P.nch++] = d.joints[j].child;
  }
  for (int b = 0; b < ty.nb; ++b) {
    int r = b;
    while (tab.body[t][r].parent >= 0) r = tab.body[t][r].parent;
    tab.body[t][b].root = r;
    ty.max_children = std::max(ty.max_children, tab.body[t][b].nch);
  }
  // contacts are generated body by body, so each body's are contiguous
  for (int b = 0; b < ty.nb; ++b) {
    int c0 = -1, c1 = -1;
    for (int c = 0; c < ty.nc; ++c)
      if (d.contacts[c].body == b) {
        if (c0 < 0) c0 = c;
        c1 = c + 1;
      }
    tab.body[t][b].c0 = c0 < 0 ? 0 : c0;
    tab.body[t][b].c1 = c0 < 0 ? 0 : c1;
    ty.max_contacts = std::max(ty.max_contacts, tab.body[t][b].c1 - tab.body[t][b].c0);
  }
  for (int c = 0; c < ty.nc; ++c) {
    ContactT& C = tab.contact[t][c];
    C.body = d.contacts[c].body;
    for (int k = 0; k < 3; ++k) C.l[k] = (float)d.contacts[c].l[k];
    C.rho = (float)d.contacts[c].rho;
  }
  // body-body candidates and the lane that evaluates each
  ty.np = (int)d.pairs.size();
  for (int c = 0; c < ty.np; ++c) {
    const PairD& S = d.pairs[c];
    PairT& P = tab.pair[t][c];
    P = PairT{};
    P.a = S.a;
    P.b = S.b;
    P.kind = S.kind;
    auto frozen3 = [](const double* f) { return f[0] == 0 && f[1] == 0 && f[2] == 0; };
    P.rot_a = frozen3(d.bodies[S.a].free_r) ? 0 : 1;
    P.rot_b = frozen3(d.bodies[S.b].free_r) ? 0 : 1;
    P.im_a = frozen3(d.bodies[S.a].free_p) ? 0.f : (float)(1.0 / d.bodies[S.a].mass);
    P.im_b = frozen3(d.bodies[S.b].free_p) ? 0.f : (float)(1.0 / d.bodies[S.b].mass);
    P.ra = (float)S.ra;
    P.rb = (float)S.rb;
    for (int k = 0; k < 3; ++k) {
      P.a0[k] = (float)S.a0[k];
      P.a1[k] = (float)S.a1[k];
      P.b0[k] = (float)S.b0[k];
      P.b1[k] = (float)S.b1[k];
      P.ah[k] = (float)S.ah[k];
      P.bh[k] = (float)S.bh[k];
    }
    for (int k = 0; k < 9; ++k) {
      P.aR[k] = (float)S.aR[k];
      P.bR[k] = (float)S.bR[k];
      if (S.aR[k] != (k % 4 == 0 ? 1.0 : 0.0) || S.bR[k] != (k % 4 == 0 ? 1.0 : 0.0)) P.box_rot = 1;
    }
    // origins farther apart than the two features' extents from their
    // origins plus the radii cannot be in contact
    auto norm = [](const double* v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
    auto extent = [&](bool box, const double* p0, const double* p1, const double* half, double r) {
      return box ? norm(p0) + norm(half) : std::max(norm(p0), norm(p1)) + r;
    };
    const bool box_a = S.kind == PK_BP || S.kind == PK_BS, box_b = S.kind == PK_PB || S.kind == PK_SB;
    const double reach = extent(box_a, S.a0, S.a1, S.ah, S.ra) + extent(box_b, S.b0, S.b1, S.bh, S.rb);
    // with a margin (0.01% and 0.1 mm) far above the FP32 rounding of positions and of the test
    P.reach = (float)(reach * (1.0 + 1e-4) + 1e-4);
    // the bound test: a segment side is the line (the first body's when both
    // are), the other side a ball around its feature's centre: a box's centre
    // with its half diagonal, a segment's midpoint with its half length, or
    // a point; a contact needs the line within both radii plus that extent
    {
      const bool seg_a = S.kind == PK_SP || S.kind == PK_SS || S.kind == PK_SB;
      const bool seg_b = S.kind == PK_PS || S.kind == PK_BS;
      const bool line_b = seg_b || S.kind == PK_BP;  // otherwise the first body's feature is the line
      const double* l0 = line_b ? S.b0 : S.a0;
      const double* l1 = line_b ? S.b1 : S.a1;
      const bool lseg = line_b ? seg_b : seg_a;
      const bool kbox = line_b ? box_a : box_b;
      const double* k0 = line_b ? S.a0 : S.b0;
      const double* k1 = line_b ? S.a1 : S.b1;
      const double* kh = line_b ? S.ah : S.bh;
      const bool kseg = line_b ? (S.kind == PK_SS) : (S.kind == PK_PS || S.kind == PK_SS);
      double kcen[3], ext = 0.0;
      for (int k = 0; k < 3; ++k) kcen[k] = kseg ? 0.5 * (k0[k] + k1[k]) : k0[k];
      if (kbox) ext = norm(kh);
      if (kseg) {
        const double dk[3] = {k1[0] - k0[0], k1[1] - k0[1], k1[2] - k0[2]};
        ext = 0.5 * norm(dk);
      }
      const double rt = (S.ra + S.rb + ext) * (1.0 + 1e-4) + 1e-4;
      for (int k = 0; k < 3; ++k) {
        P.lo[k] = (float)l0[k];
        P.ld[k] = lseg ? (float)(l1[k] - l0[k]) : 0.f;
        P.kc[k] = (float)kcen[k];
      }
      P.lo[3] = (float)(rt * rt);
      P.ld[3] = 0.f;
      P.kc[3] = line_b ? 1.f : 0.f;
    }
    BodyT& A = tab.body[t][S.a];
    BodyT& Bb = tab.body[t][S.b];
    A.pairs[A.npair++] = c;
    Bb.pairs[Bb.npair++] = c;
    BodyT& H = tab.body[t][S.handler];
    const int slot = H.nh;  // within MAXH and MAXR: checked when the description was built
    H.hp[H.nh++] = c;
    A.recva[slot] |= (uint32_t)S.handler << (4 * A.nra[slot]);
    ++A.nra[slot];
    Bb.recvb[slot] |= (uint32_t)S.handler << (4 * Bb.nrb[slot]);
    ++Bb.nrb[slot];
  }
  for (int b = 0; b < ty.nb; ++b) {
    const BodyT& B = tab.body[t][b];
    ty.max_handled = std::max(ty.max_handled, B.nh);
    for (int i = 0; i < MAXH; ++i) {
      ty.recv_na[i] = std::max(ty.recv_na[i], B.nra[i]);
      ty.recv_nb[i] = std::max(ty.recv_nb[i], B.nrb[i]);
    }
  }
  int dof0 = 0;
  for (int j = 0; j < ty.nj; ++j) {
    const JointD& S = d.joints[j];
    JointT& J = tab.joint[t][j];
    J = JointT{};
    J.parent = S.parent;
    J.child = S.child;
    J.dof = S.dof;
    J.dof0 = dof0;
    dof0 += S.dof;
    for (int k = 0; k < 3; ++k) {
      J.ap[k] = (float)S.ap[k];
      J.ac[k] = (float)S.ac[k];
      J.lo[k] = (float)S.lo[k];
      J.hi[k] = (float)S.hi[k];
      J.act[k] = -1;
      J.gear[k] = 0.f;
      J.act_lo[k] = -1.f;
      J.act_hi[k] = 1.f;
      J.act_pd[k] = 0.f;
      double def = (k < S.dof && !(S.lo[k] <= 0.0 && 0.0 <= S.hi[k])) ? 0.5 * (S.lo[k] + S.hi[k]) : 0.0;
      J.def_angle[k] = (float)def;
    }
    for (int k = 0; k < 9; ++k) {
      J.FP[k] = (float)S.FP[k];
      J.FC[k] = (float)S.FC[k];
    }
    J.k_lin = (float)S.k_lin;
    J.c_lin = (float)S.c_lin;
    J.k_ang = (float)S.k_ang;
    J.c_ang = (float)S.c_ang;
    J.k_lim = (float)S.k_lim;
    ty.max_dof = std::max(ty.max_dof, S.dof);
  }
  for (int a = 0; a < ty.na; ++a) {
    JointT& J = tab.joint[t][d.actions[a].joint];
    const int k = d.actions[a].axis;
    J.act[k] = a;
    J.gear[k] = (float)d.actions[a].gear;
    if (d.actions[a].mode == 1) {  // target angle: clamped to the joint's range, drives theta towards it
      J.act_lo[k] = J.lo[k];
      J.act_hi[k] = J.hi[k];
      J.act_pd[k] = 1.f;
    }
  }
  // contact lanes of the fused forward without a tape: a body with more
  // than two ground-contact candidates takes ceil(n / 2) - 1 extra lanes
  // (copies of its entry, which integrate the same state), each evaluating
  // two of its candidates, so that a wavefront evaluates at most two
  // candidate slots per substep; a type whose contact lanes would not fit
  // (MAXB lanes, 8 per group) keeps every candidate on its body's lane
  ty.nl = ty.nb;
  ty.max_lc = ty.max_contacts;
  ty.max_ng = 1;
  for (int b = 0; b < ty.nb; ++b) {
    BodyT& B = tab.body[t][b];
    B.l0 = B.c0;
    B.l1 = B.c1;
    B.body_of = b;
    B.ng = 1;
    B.grp_packed = (uint32_t)b;
  }
  {
    int extra = 0, max_ng = 1;
    for (int b = 0; b < ty.nb; ++b) {
      const int n = tab.body[t][b].c1 - tab.body[t][b].c0;
      const int g = n > 2 ? (n + 1) / 2 : 1;
      extra += g - 1;
      max_ng = std::max(max_ng, g);
    }
    if (extra > 0 && ty.nb + extra <= MAXB && max_ng <= 8) {
      int lane = ty.nb;
      ty.max_lc = 0;
      for (int b = 0; b < ty.nb; ++b) {
        BodyT& B = tab.body[t][b];
        const int n = B.c1 - B.c0;
        if (n > 2) {
          const int g = (n + 1) / 2;
          B.l1 = B.c0 + 2;
          B.ng = g;
          for (int i = 1; i < g; ++i) B.grp_packed |= (uint32_t)(lane + i - 1) << (4 * i);
          for (int i = 1; i < g; ++i) {
            BodyT& M = tab.body[t][lane + i - 1];
            M = B;  // same constants, joint, children and body-body share lists
            M.l0 = B.c0 + 2 * i;
            M.l1 = std::min(B.c1, M.l0 + 2);
            M.nh = 0;  // evaluates no body-body candidate
            for (int k = 0; k < MAXH; ++k) M.hp[k] = 0;
          }
          lane += g - 1;
        }
        ty.max_lc = std::max(ty.max_lc, B.l1 - B.l0);
      }
      for (int m = ty.nb; m < lane; ++m) ty.max_lc = std::max(ty.max_lc, tab.body[t][m].l1 - tab.body[t][m].l0);
      ty.nl = lane;
      ty.max_ng = max_ng;
    }
  }

  // parent-before-child order
  int n = 0;
  std::vector<int> placed(ty.nb, 0);
  while (n < ty.nb) {
    for (int b = 0; b < ty.nb; ++b) {
      if (placed[b]) continue;
      int p = tab.body[t][b].parent;
      if (p < 0 || placed[p]) {
        tab.topo[t][n++] = b;
        placed[b] = 1;
      }
    }
  }
}

}  // namespace bx
